/*
 * ddf.h -- C ABI of libddf.so: the directional-distance-field (DDF) hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow "Neural directional distance field object representation
 * for uni-directional path-traced rendering" (Behera and Mishra, arXiv 2306.16142):
 *   - the field phi(x, theta): distance from a point x along a direction theta to
 *     the surface, infinite when the ray misses (Sec. III-A);
 *   - its neural form MLP_w(x, theta) (Sec. IV-A), evaluated here on batches of rays;
 *   - the gradient of the field with respect to the query point, which gives the
 *     surface normal (Eq. 3, Sec. IV-B);
 *   - the ground-truth labels from ray shooting against the triangle mesh by a
 *     linear search over all triangles (Sec. I, Sec. VI-B) with the odd-even
 *     inside rule (Sec. V-B);
 *   - the path tracer whose nearest-hit search the field replaces (Fig. 1);
 *   - the informative training-data sampler built on the ray shooting (Sec. V-B);
 *   - the unsigned distance field as the minimum of the field over directions (Eq. 5);
 *   - training with the paper's clamp / squish losses (Eqs. 6-7) and the directed Eikonal
 *     property of the field (Eq. 2) as a penalty.
 *
 * Conventions common to every entry point
 *   Memory    Every array argument is DEVICE memory owned by the caller unless the
 *             comment says "host".  The library never allocates, frees or keeps
 *             caller memory; scratch comes from a caller-supplied workspace whose
 *             size the matching *_workspace_size call returns (ddf_udf_noalloc alone
 *             uses a fixed scratch array of the library's instead).
 *   Layout    Ray batches are structure-of-arrays float32: an array "[k][n]" holds
 *             row r of ray i at index r*n + i.  Triangles are a "[9][m]" soup of
 *             corners v0xyz, v1xyz, v2xyz.
 *   Streams   `stream` is a hipStream_t (NULL = the null stream).  Calls only
 *             enqueue work; outputs are valid once the stream has synchronised.
 *             No call synchronises the host, so every call may be captured in a
 *             HIP graph (those needing a workspace clear it with kernels).
 *   Errors    Arguments are validated before anything is enqueued.  On error
 *             nothing is launched, a non-zero ddf_status is returned and
 *             ddf_last_error() returns a thread-local message.  n == 0 is a no-op,
 *             except where a loss is formed: ddf_loss_seeds(_ex), ddf_train_step(_chunked,
 *             _ex, _eikonal) and ddf_paper_train_step reject an empty batch with
 *             INVALID_ARG (the mean loss of no rays is undefined, and an Adam step on it
 *             would still move the parameters).  No C++ exception crosses this boundary.
 */
#ifndef DDF_H
#define DDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ddf_status;
#define DDF_OK 0
#define DDF_ERR_INVALID_ARG 1
#define DDF_ERR_UNSUPPORTED 2
#define DDF_ERR_WORKSPACE 3
#define DDF_ERR_HIP 4

typedef void *ddf_stream;   /* hipStream_t */

/* Arithmetic of the network's layer products (accumulation is always float32). */
#define DDF_PREC_FP32 0
#define DDF_PREC_BF16 1
#define DDF_PREC_FP8 2      /* OCP e4m3fn operands, static per-layer scales */

/* Network shape: `depth` hidden ReLU layers of `width` units on the 65 Fourier
 * features of the ray (ox, oy, oz, theta, phi), then a 2-unit affine head
 * (hit logit, distance).  Supported widths: 128 and 256; depth 1..8. */
typedef struct {
    int32_t width;
    int32_t depth;
    int32_t precision;      /* DDF_PREC_* */
    const void *packed;     /* device blob written by ddf_pack_net for this shape/precision */
} ddf_net;

/* Library version of this header (DDF_ABI_VERSION). */
#define DDF_ABI_VERSION 1
int32_t ddf_abi_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char *ddf_last_error(void);

/* ---------------------------------------------------------------- labeller
 * Nearest hit of each ray against every triangle (linear search; Sec. I, ray
 * shooting for labels Sec. VI-B), two-sided Moller-Trumbore, edges inclusive,
 * accepted when t_min < t < t_max; ties go to the lowest triangle index.
 *   orig, dir    [3][n] ray origins and directions (any non-zero length; t is in
 *                units of |dir|).
 *   tris         [9][m] triangle corners.
 *   t_out        [n] nearest t, +inf on a miss (also for NaN rays).
 *   tri_out      [n] index of the nearest triangle, -1 on a miss.
 *   crossings    [n] number of accepted hits (odd-even inside rule, Sec. V-B),
 *                or NULL.
 * Decisions are taken in float32 with a forward error bound; a test whose
 * outcome the bound cannot settle (near an edge, near grazing, near t_min /
 * t_max) is re-evaluated in float64 from the same float32 inputs.
 * Errors: INVALID_ARG for n < 0, m < 0, NULL arrays with n > 0, t_min >= t_max. */
ddf_status ddf_label_rays(const float *orig, const float *dir, int64_t n,
                          const float *tris, int64_t m, float t_min, float t_max,
                          float *t_out, int32_t *tri_out, uint32_t *crossings,
                          ddf_stream stream);

/* ---------------------------------------------------------------- rays
 * Ray assembly (Eq. 1 inverted): rays_out [5][n] = (ox, oy, oz, theta, phi) with
 * theta = polar angle of dir from +z in [0, pi] and phi = atan2(dy, dx) wrapped
 * into [0, 2 pi) (0 on the z axis).  orig, dir [3][n].  In place is not allowed. */
ddf_status ddf_assemble_rays(const float *orig, const float *dir, int64_t n, float *rays_out,
                             ddf_stream stream);

/* ---------------------------------------------------------------- training-data sampler
 * The informative sampler of Sec. V-B (Eqs. 8-12, Fig. 2) on top of the labeller.
 * For each face f in face_first .. face_first + n_faces - 1 (of the m triangles):
 *   s_fc points (1 - a - b) p0 + a p1 + b p2 (Eq. 8), (a, b) folded to (1 - a, 1 - b)
 *     when a + b > 1 (decided exactly), from face_uv [2][m * s_fc] (column f * s_fc + j);
 *   s_dr directions of polar angle a pi and azimuth 2 b pi (Eq. 9; Eq. 1 for the
 *     vector), from dir_uv [2][m * s_dr] (column f * s_dr + j), shared by the face's points.
 * Pair (point, direction) i = (f - face_first) * s_fc * s_dr + point * s_dr + direction.
 * A pair is kept when its ray meets no triangle at t > eps (eps steps over the point's own
 * face; on a closed mesh a ray into the solid always meets another face, so this also drops
 * what the odd-even rule calls inside) and the point lies inside the cube [-1, 1]^3.
 * A kept ray is marched to where it leaves the cube, t_k = k t_exit / s_p, k = 1..s_p, and at
 * q = p + t_k d it yields, in this order:
 *   (q, -d; t_k)      looking back at the face point (Eq. 10);
 *   (q,  d; +inf)     looking on along the ray (Eq. 11);
 *   (q, polar + pi/2; +inf) and (q, polar - pi/2; +inf), each only when that ray meets no
 *                     triangle (Eq. 12).
 * Samples are ordered by pair, then k, then the order above (deterministic).
 *   rays_out  [5][cap] (qx, qy, qz, theta, phi), theta in [0, pi], phi in [0, 2 pi), row
 *             stride cap; t_out [cap] labels (+inf: no hit); pair_out [cap] source pair
 *             index, or NULL.  Samples beyond cap are counted but not written.
 *   count_out device int64: the number of samples (may exceed cap).
 *   ws        ddf_dataset_workspace_size bytes (device, caller-owned).
 * Random numbers are inputs (uniforms in [0, 1)), so a seed fixes the dataset.
 * Errors: INVALID_ARG for s_fc, s_dr or s_p < 1, eps < 0 or not finite, a face range
 * beyond m, cap < 0, NULL arrays that are needed; UNSUPPORTED when
 * n_faces * s_fc * s_dr * s_p reaches 2^29; WORKSPACE when ws is too small.
 * n_faces == 0 writes count 0 and nothing else. */
typedef struct {
    int32_t s_fc;        /* points per face (Eq. 8) */
    int32_t s_dr;        /* directions per face (Eq. 9) */
    int32_t s_p;         /* marching steps per kept ray (Eq. 10) */
    float eps;           /* offset over the own face for the kept test (scene units) */
    int64_t face_first;  /* first sampled face */
    int64_t n_faces;     /* number of sampled faces (every triangle is still intersected) */
} ddf_dataset_params;

ddf_status ddf_dataset_workspace_size(const ddf_dataset_params *p, size_t *bytes);
ddf_status ddf_sample_dataset(const float *tris, int64_t m, const ddf_dataset_params *p, const float *face_uv,
                              const float *dir_uv, float *rays_out, float *t_out, int32_t *pair_out, int64_t cap,
                              int64_t *count_out, void *ws, size_t ws_bytes, ddf_stream stream);

/* ---------------------------------------------------------------- unsigned distance field
 * UDF(x) = min over a direction set of phi(x, theta) (Sec. III-A, Eq. 5), with phi the
 * network's distance where logit > 0 and +inf where it reports a miss (a NaN distance counts
 * as a miss).
 *   points   [3][n_points] query points (network inputs as given: inside the domain).
 *   dirs     [3][n_dirs] unit directions, turned into the network's angles as
 *            ddf_assemble_rays does.
 *   udf_out  [n_points] the minimum, +inf where every direction misses (or n_dirs == 0).
 *   arg_out  [n_points] the lowest direction index reaching it, -1 where none; or NULL.
 *   ws       workspace; ddf_udf_workspace_size gives the size for one pass over up to
 *            2^24 queries; a smaller workspace (at least one point's queries) is used in
 *            chunks of points, with the same results.
 * Any network ddf_forward accepts.  Errors: INVALID_ARG for negative sizes, NULL arrays that
 * are needed; UNSUPPORTED for unsupported networks or n_dirs >= 2^31; WORKSPACE when ws
 * cannot hold one point's queries.  n_points == 0 is a no-op. */
ddf_status ddf_udf_workspace_size(int64_t n_points, int64_t n_dirs, size_t *bytes);
ddf_status ddf_udf(const ddf_net *net, const float *points, int64_t n_points, const float *dirs, int64_t n_dirs,
                   float *udf_out, int32_t *arg_out, void *ws, size_t ws_bytes, ddf_stream stream);

/* ddf_udf for callers that cannot allocate memory (code under HIP graph capture, serving loops
 * and harnesses that forbid hipMalloc): no workspace argument, and no allocation of any kind.
 * Its scratch is a fixed 8 MiB array in device memory, one per GPU the library runs on, held
 * until the process ends; its address is looked up once per device on the first call there.
 * The same kernels and results as ddf_udf (bit for bit): the fused form while the keys of all
 * points fit (up to about a million points), otherwise chunks of points as ddf_udf does with a
 * small workspace.  Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other threads, other streams) race and must be serialised by the caller; nothing is
 * assumed about the array's previous contents (the keys are reset by a kernel).
 * Errors: those of ddf_udf, plus UNSUPPORTED for n_dirs > 65536 (one point's queries must fit
 * the scratch) and HIP_ERROR when the scratch's address cannot be obtained. */
ddf_status ddf_udf_noalloc(const ddf_net *net, const float *points, int64_t n_points, const float *dirs,
                           int64_t n_dirs, float *udf_out, int32_t *arg_out, ddf_stream stream);

/* ---------------------------------------------------------------- launch tuning
 * Process-wide launch-shape knobs.  They decide how work is spread over the GPU and
 * never change a result (each candidate gives bit-identical outputs); an autotuner times
 * the candidates on a workload and keeps the fastest.  Read when a call launches its
 * kernels: change knobs between calls, not while another thread is inside a call.
 * Invalid knob or value: DDF_ERR_INVALID_ARG, nothing changes. */
#define DDF_TUNE_STREAM_WG_PER_CU 0     /* workgroups per CU of the streamed bf16 network kernel:
                                           1 or 2 (2 applies where registers and LDS allow it,
                                           that is width 128); default 2 */
#define DDF_TUNE_CULL_RAYS_PER_BLOCK 1  /* rays per block of the multi-object instance culling:
                                           power of two in [256, 16384]; default 2048 */
#define DDF_TUNE_GRAD_WG_PER_CU 2       /* workgroups per CU of the per-wave gradient kernel (input
                                           gradients; the float32 training sweep sizes its own
                                           grid): 1, 2 or 4; default 2 */
#define DDF_TUNE_COUNT 3
ddf_status ddf_set_tuning(int32_t knob, int32_t value);
ddf_status ddf_get_tuning(int32_t knob, int32_t *value);

/* ---------------------------------------------------------------- network
 * Size in bytes of the packed blob for a shape and precision. */
ddf_status ddf_packed_bytes(int32_t width, int32_t depth, int32_t precision, size_t *bytes);

/* Packs the flat float32 parameters (device; per affine layer the weight
 * [out][in] row-major then the bias [out], the order of torch.nn.Linear) into the
 * MFMA-tile blob of `precision`.  For DDF_PREC_FP8, `scales` (device, [2*(depth+1)]:
 * weight scale and input scale per affine layer, each a positive power of two, as
 * ddf_fp8_scales returns them) is required; otherwise it must be NULL.  A forward of
 * an fp8 blob whose scales are not powers of two writes NaN.  packed: device buffer
 * of ddf_packed_bytes bytes. */
ddf_status ddf_pack_net(const float *params, int32_t width, int32_t depth, int32_t precision,
                        const float *scales, void *packed, ddf_stream stream);

/* Static fp8 scales from a float32 network: per affine layer, the smallest power of
 * two s with absmax / s <= 448 for the weight and for its input over the calibration
 * rays (power-of-two scales make every rescaling between layers exact, so the
 * kernels apply it through the MFMA's operand scale).  net_fp32 must be a
 * DDF_PREC_FP32 blob of the same parameters.  calib [5][n_calib]; scales_out
 * device [2*(depth+1)]. */
ddf_status ddf_fp8_scales(const ddf_net *net_fp32, const float *params, const float *calib,
                          int64_t n_calib, float *scales_out, ddf_stream stream);

/* Batched network query (Sec. IV-A, MLP_w(x, theta)): rays [5][n] ->
 * logit_out [n] (hit <=> logit > 0) and dist_out [n] (meaningful on hits).
 * NaN rays give NaN outputs. */
ddf_status ddf_forward(const ddf_net *net, const float *rays, int64_t n,
                       float *logit_out, float *dist_out, ddf_stream stream);

/* The same query straight from origins orig [3][n] and unit directions dir [3][n] (device,
 * float32, row r of ray i at r * n + i): ray assembly (as ddf_assemble_rays, Eq. 1 read
 * backwards) and the network in one kernel, results bit-identical to ddf_assemble_rays
 * followed by ddf_forward.  Needs a bf16 or fp8 network whose packed weights fit in one
 * CU's LDS (width 128, depth <= 4); other networks: DDF_ERR_UNSUPPORTED. */
ddf_status ddf_query(const ddf_net *net, const float *orig, const float *dir, int64_t n, float *logit_out,
                     float *dist_out, ddf_stream stream);

/* ---------------------------------------------------------------- gradients
 * Reverse-mode gradient of sum(g_logit * logit + g_dist * dist) over the batch.  The
 * input gradient's origin part is the derivative of the field with respect to the
 * query point that gives the surface normal (Eq. 3; Sec. IV-B takes it by automatic
 * differentiation); the parameter gradient is the training backward (Sec. V-A).
 *   net       DDF_PREC_FP32, or DDF_PREC_BF16 when g_params is NULL.
 *   rays      [5][n]; g_logit, g_dist [n] seeds (either may be NULL = zeros).
 *   g_rays    [5][n] d/d(ox, oy, oz, theta, phi), or NULL.
 *   g_params  [P] float32 in the flat parameter order, or NULL.  Written, or added to
 *             when flags has DDF_GRAD_ACCUMULATE.  Needs the workspace of
 *             ddf_train_workspace_size(width, depth, n); with g_params NULL no
 *             workspace is used (ws may be NULL).
 * The forward pass is recomputed inside the kernel (ReLU masks kept on chip); the
 * parameter gradient sums over rays in fixed-size chunks combined in a fixed order, so
 * repeated calls give bitwise identical results. */
#define DDF_GRAD_ACCUMULATE 1u
ddf_status ddf_train_workspace_size(int32_t width, int32_t depth, int64_t n, size_t *bytes);
ddf_status ddf_backward(const ddf_net *net, const float *rays, int64_t n, const float *g_logit,
                        const float *g_dist, float *g_rays, float *g_params, uint32_t flags,
                        void *ws, size_t ws_bytes, ddf_stream stream);

/* Loss of the training labels and its seeds: binary cross-entropy with logits on the hit
 * flag (hit <=> t_label < +inf), mean over the n rays, plus the L1 distance error
 * |dist - t_label| averaged over hit rays (weights 1:1).  g_logit = (sigmoid(logit) -
 * hit) / n; g_dist = sign(dist - t) / n_hit on hits, 0 elsewhere.  loss_out: device
 * scalar.  ws: device scratch of at least 4160 bytes. */
ddf_status ddf_loss_seeds(const float *logit, const float *dist, const float *t_label, int64_t n,
                          float *g_logit, float *g_dist, float *loss_out, void *ws, size_t ws_bytes,
                          ddf_stream stream);

/* One Adam update (Kingma and Ba; Sec. V-A optimises with Adam) of `count` float32
 * parameters with bias correction for the 1-based `step`; no weight decay. */
ddf_status ddf_adam_step(float *params, const float *grads, float *m, float *v, int64_t count,
                         int64_t step, float lr, float beta1, float beta2, float eps, ddf_stream stream);

/* One training step on a labelled batch: loss seeds, parameter gradients (as
 * ddf_backward), Adam (beta 0.9 / 0.999, eps 1e-8) on `params` / `adam_m` / `adam_v`, and
 * repacking of `net` (a DDF_PREC_FP32 blob of `params`, rewritten in place).
 *   rays [5][n], t_label [n] (+inf = miss); loss_out: device scalar (loss before the
 *   update); g_params [P] receives the gradient; ws: ddf_train_workspace_size bytes. */
ddf_status ddf_train_step(const ddf_net *net, float *params, float *adam_m, float *adam_v,
                          int64_t step, float lr, const float *rays, const float *t_label, int64_t n,
                          float *loss_out, float *g_params, void *ws, size_t ws_bytes,
                          ddf_stream stream);

/* The same training step for a batch whose workspace would be too large: the n rays are
 * swept in column ranges of `chunk` rays, each recomputing its forward pass and keeping its
 * activations only in a workspace of ddf_train_workspace_size(width, depth, chunk) bytes
 * (memory independent of n).  The loss and its seeds use the whole batch's normalisation
 * (1 / n, 1 / hits), so the gradient is that of the full batch, summed over chunks in a
 * fixed order (equal to ddf_train_step's up to float32 summation order); then one Adam
 * update and repack.  rays [5][n] and t_label [n] as in ddf_train_step; chunk >= 1
 * (values above n mean one chunk). */
ddf_status ddf_train_step_chunked(const ddf_net *net, float *params, float *adam_m, float *adam_v,
                                  int64_t step, float lr, const float *rays, const float *t_label,
                                  int64_t n, int64_t chunk, float *loss_out, float *g_params, void *ws,
                                  size_t ws_bytes, ddf_stream stream);

/* Training losses (the default is the one above):
 *   DDF_LOSS_BCE_L1  binary cross-entropy on the hit logit + L1 on hit distances (1:1);
 *   DDF_LOSS_CLAMP   the clamp loss of Eq. 7 (Sec. V-A) on the distance output alone:
 *                    |c(t) - c(dist)| / n with c the two-sided clamp at `delta` (> 0,
 *                    finite); a miss (t = +inf) clamps to delta;
 *   DDF_LOSS_SQUISH  the squish loss of Eq. 6 (Sec. IV-A) on the distance alone, read with
 *                    the absolute value and sigma = tanh: |tanh(t) - tanh(dist)| / n,
 *                    tanh(+inf) = 1 (delta unused).
 * With the clamp and squish losses g_logit is 0 and g_dist = sign(c(dist) - c(t)) c'(dist) / n
 * (c' = 1 strictly inside the clamp window and 0 outside or on its edges; 1 - tanh^2). */
#define DDF_LOSS_BCE_L1 0
#define DDF_LOSS_CLAMP 1
#define DDF_LOSS_SQUISH 2
typedef struct {
    int32_t kind;   /* DDF_LOSS_* */
    float delta;    /* clamp window of DDF_LOSS_CLAMP */
} ddf_loss;

/* ddf_loss_seeds with a chosen loss (`loss` NULL: DDF_LOSS_BCE_L1).  Errors as
 * ddf_loss_seeds, plus INVALID_ARG for an unknown kind or a clamp without a finite delta > 0. */
ddf_status ddf_loss_seeds_ex(const float *logit, const float *dist, const float *t_label, int64_t n,
                             const ddf_loss *loss, float *g_logit, float *g_dist, float *loss_out, void *ws,
                             size_t ws_bytes, ddf_stream stream);

/* The training step with a chosen loss: chunk == 0 is ddf_train_step, chunk >= 1 is
 * ddf_train_step_chunked (same workspace rules); `loss` NULL: DDF_LOSS_BCE_L1.  Errors as
 * those two, plus INVALID_ARG for a bad loss or a negative chunk. */
ddf_status ddf_train_step_ex(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step,
                             float lr, const float *rays, const float *t_label, int64_t n, int64_t chunk,
                             const ddf_loss *loss, float *loss_out, float *g_params, void *ws, size_t ws_bytes,
                             ddf_stream stream);

/* A training step with the directed Eikonal penalty of Eq. 2 (Sec. III-A): along its own ray
 * the field falls at unit rate (grad_x phi . d = -1 where the ray hits).  The derivative is
 * taken as a forward difference along the ray, r = (phi(x + h d) - phi(x)) / h + 1, and the
 * loss is `loss`'s (NULL: DDF_LOSS_BCE_L1) on the rays plus lambda / n * sum r^2 over rays
 * whose label is a hit farther than h.  The batch is doubled internally (the rays at their
 * origins and moved by h along their unit direction, each ray and its moved copy in the same
 * 64-column tile of the training sweep), so the gradient needs first-order passes only: one
 * sweep forms both outputs of every pair, the pair's loss and penalty seeds in its workgroup,
 * and the adjoints; then the weight-gradient products, Adam, repack.
 *   orig, dir [3][n] origins and directions (any non-zero length; normalised for the move);
 *   t_label [n] labels (+inf = miss); loss_out: device scalar (both terms, before the update);
 *   ws: ddf_eikonal_workspace_size(width, depth, n) bytes: the doubled batch is swept whole
 *   (activations of 2 n rays (n rounded up to 32), about (65 + 2 depth width) x 8 n bytes;
 *   there is no chunked form).
 * Float32 networks only.  Errors: INVALID_ARG for a bad argument, h <= 0 or not finite,
 * lambda < 0 or not finite, a bad loss; WORKSPACE when ws is too small. */
ddf_status ddf_eikonal_workspace_size(int32_t width, int32_t depth, int64_t n, size_t *bytes);
ddf_status ddf_train_step_eikonal(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step,
                                  float lr, const float *orig, const float *dir, const float *t_label, int64_t n,
                                  float h, float lambda, const ddf_loss *loss, float *loss_out, float *g_params,
                                  void *ws, size_t ws_bytes, ddf_stream stream);

/* ---------------------------------------------------------------- the paper's network
 * The network of Sec. V-A as the paper builds it: `depth` (the paper: 8) weight-normalised
 * hidden ReLU layers of 512 units on the raw oriented point (ox, oy, oz, polar angle,
 * azimuth; Sec. IV-A, MLP_w : (R^3, R^2) -> R), then one affine output, the field value.
 * Dropout (p = 0.5 in the paper) is the identity when the network is queried; the training
 * step applies it (ddf_paper_train_step).  Weight normalisation (Salimans and Kingma 2016): W_l = g_l v_l / |v_l| per
 * output row, folded on the device by ddf_paper_pack (every row of v_l must be non-zero).
 *   Parameters (float32, flat, device): per hidden layer l = 0 .. depth - 1: v_l [512][in_l]
 *   row-major (in_0 = 5, else 512), g_l [512], b_l [512]; then the output row [512] and its
 *   bias [1] (ddf_paper_param_count values).
 * Precisions: DDF_PREC_FP32 (queries, gradients, training) and DDF_PREC_BF16 (queries and
 * input gradients: the first layer takes the raw inputs in float32, the hidden layers bf16
 * operands with float32 accumulation, the output row as a bf16 pair).  depth 1..8. */
#define DDF_PAPER_WIDTH 512
typedef struct {
    int32_t depth;
    int32_t precision;      /* DDF_PREC_FP32 or DDF_PREC_BF16 */
    const void *packed;     /* device blob written by ddf_paper_pack for this depth / precision */
} ddf_paper_net;

ddf_status ddf_paper_param_count(int32_t depth, int64_t *count);
/* Bytes of the packed blob (device memory the caller allocates). */
ddf_status ddf_paper_packed_bytes(int32_t depth, int32_t precision, size_t *bytes);
/* Folds the weight normalisation and packs `params` (device, layout above) for `precision`. */
ddf_status ddf_paper_pack(const float *params, int32_t depth, int32_t precision, void *packed, ddf_stream stream);

/* Query (Sec. IV-A): rays [5][n] (ox, oy, oz, theta, phi) -> dist_out [n], the field value
 * (the paper's losses saturate misses at their clamp or squish limit).  NaN rays give NaN.
 * Errors: INVALID_ARG for NULL arrays with n > 0 or n < 0; UNSUPPORTED for a bad depth or
 * precision. */
ddf_status ddf_paper_forward(const ddf_paper_net *net, const float *rays, int64_t n, float *dist_out,
                             ddf_stream stream);

/* Reverse mode of sum(g_dist * dist) (g_dist [n], NULL = zeros); `params` are the parameters
 * `net` was packed from (needed with g_params: the weight normalisation's gradient depends on
 * v and g, not only on the folded weights; may be NULL otherwise):
 *   g_rays   [5][n] d/d(ox, oy, oz, theta, phi), or NULL; its origin part is the gradient of the
 *            field with respect to the query point that gives the normal (Eq. 3, Sec. IV-B);
 *   g_params [P] float32 in the parameter order above (gradients of v, g, b of every hidden
 *            layer through the weight normalisation, then of the output row and bias), or
 *            NULL; float32 networks only; written, or added to with DDF_GRAD_ACCUMULATE;
 *            needs ddf_paper_workspace_size(depth, n) bytes of workspace (ws unused otherwise).
 * The forward pass is recomputed inside the kernels; sums over rays run in fixed-size chunks
 * combined in a fixed order (repeated calls are bitwise identical). */
ddf_status ddf_paper_workspace_size(int32_t depth, int64_t n, size_t *bytes);
ddf_status ddf_paper_backward(const ddf_paper_net *net, const float *params, const float *rays, int64_t n,
                              const float *g_dist, float *g_rays, float *g_params, uint32_t flags, void *ws,
                              size_t ws_bytes, ddf_stream stream);

/* One training step of Sec. V-A on a labelled batch: the loss (`loss`: DDF_LOSS_CLAMP, Eq. 7,
 * or DDF_LOSS_SQUISH, Eq. 6; the paper trains on the clamp loss) on the distance of the
 * network with dropout `dropout` (the paper: 0.5; 0 = none) after every hidden ReLU, its
 * gradient with respect to every parameter, one Adam update (beta 0.9 / 0.999, eps 1e-8,
 * 1-based `step`) of `params` / `adam_m` / `adam_v`, and repacking of `net` (a DDF_PREC_FP32
 * blob of `params`, rewritten in place).
 *   Dropout is inverted (kept units scaled by 1 / (1 - dropout)); its keep decisions are a
 *   counter-based draw, so both sweeps see the same masks without storing them: with H(x)
 *   the first output of SplitMix64 from state x (Steele, Lea and Flood 2014), hidden layer l
 *   has K = H(H(H(dropout_seed) ^ step) ^ l), and unit u of ray r (0-based in the batch) is
 *   kept when the top 24 bits of H(K ^ (u << 32 | r)), read as a fraction of 2^24, are
 *   >= dropout.
 *   rays [5][n], t_label [n] (+inf = miss); loss_out: device scalar (before the update);
 *   g_params [P] receives the gradient; ws: ddf_paper_workspace_size(depth, n) bytes.
 * Errors: INVALID_ARG for a bad argument, a loss other than clamp / squish or a dropout
 * outside [0, 1); WORKSPACE. */
ddf_status ddf_paper_train_step(const ddf_paper_net *net, float *params, float *adam_m, float *adam_v, int64_t step,
                                float lr, const float *rays, const float *t_label, int64_t n, const ddf_loss *loss,
                                float dropout, uint64_t dropout_seed, float *loss_out, float *g_params, void *ws,
                                size_t ws_bytes, ddf_stream stream);

/* ---------------------------------------------------------------- renderer
 * Wavefront path tracer of Fig. 1 in which the nearest-hit search is either the
 * brute-force triangle search (backend MESH) or the network (backend NET): the
 * "modified path tracer" of Sec. I / Sec. IV.  Per bounce: query -> hit point and
 * normal (mesh face normal, or Eq. 3 from the network's distance gradient with respect
 * to the query point) -> next-event estimation towards one point light (shadow ray
 * query) -> cosine-weighted Lambertian scatter -> Russian roulette -> compaction of the
 * surviving paths (wave ballot + one atomic per wave).
 *
 * Readings (the paper gives no camera, light, sampler or termination rule):
 *   pinhole camera (eye, target, up, vertical field of view), pixel centre at 1 spp,
 *   otherwise a jitter from random dimensions 0, 1; network queries start at the
 *   entry of the domain cube [-1,1]^3 (t = entry + distance; hit <=> logit > 0 and t >= 0);
 *   shadow / scatter origins x + eps n; scatter by Malley's method in the basis of Duff
 *   et al. 2017; after the scatter of bounce b >= rr_start, survival probability
 *   q = min(0.95, max throughput channel).  Random numbers: SplitMix64 (Steele, Lea,
 *   Flood 2014) as a counter hash, u = (h >> 40) 2^-24 with
 *   h = H(H(H(H(H(seed) ^ pixel) ^ sample) ^ bounce) ^ dim), H(x) = SplitMix64 output of
 *   state x; dimensions 2, 3 scatter, 4 roulette.
 * Every path's radiance is kept per path and summed per pixel in sample order, so the
 * image does not depend on queue order (bitwise reproducible).                        */
#define DDF_BACKEND_MESH 0
#define DDF_BACKEND_NET 1
#define DDF_BACKEND_MULTI 2     /* several networks placed as rigid instances */

/* One rigid instance of a network: x_world = R x_object + T.  Each network's domain is the
 * cube [-1,1]^3 of its object space; rays are moved into object space, queried from the
 * cube entry, and the nearest hit over all instances wins (distances are preserved by rigid
 * maps; ties go to the instance listed first).  Scenes of objects are the paper's stated
 * future work (Sec. VII). */
typedef struct {
    float R[9];                 /* rotation, row-major, object to world */
    float T[3];                 /* translation */
    int32_t net;                /* index into ddf_scene.nets */
} ddf_instance;

typedef struct {
    int32_t backend;            /* DDF_BACKEND_* */
    const float *tris;          /* MESH: device [9][m] */
    int64_t m;
    const ddf_net *net;         /* NET: DDF_PREC_FP32 or DDF_PREC_BF16 network (host struct) */
    int32_t n_nets;             /* MULTI: networks (host array), all float32 or all bfloat16, */
    const ddf_net *nets;        /*        at most 8 of each width */
    int32_t n_instances;        /* MULTI: instances (host array), at most 64 */
    const ddf_instance *instances;
} ddf_scene;

typedef struct {
    int32_t width, height, spp, bounces, rr_start;
    uint64_t seed;
    float eps;
    float eye[3], target[3], up[3], vfov_deg;
    float light_pos[3], light_intensity[3], albedo[3];
    int32_t spp_chunk;          /* samples per pixel traced together (0 = choose) */
} ddf_render_params;

/* Workspace bytes for a render (depends on width, height, the sample chunk and, for MULTI,
 * the number of instances). */
ddf_status ddf_render_workspace_size(const ddf_scene *scene, const ddf_render_params *p, size_t *bytes);

/* radiance [3][height][width] (mean over samples; row 0 at the top); depth [height][width]
 * and normal [3][height][width] of sample 0's primary hit (+inf / 0 on a miss) or NULL;
 * stats: device uint32, summed over chunks, or NULL: [bounces] paths entering each bounce,
 * then [bounces] shadow rays traced in each bounce (one per hit facing the light); for MESH
 * and NET followed by [bounces] hits in each bounce and [bounces] rays of each bounce's
 * nearest-hit pass (NET queries only the rays that enter the cube [-1, 1]^3, where the field
 * is defined: a ray that misses it misses the object; MESH traces every path); for MULTI by
 * [bounces][n_nets] (ray, instance) pairs queried per network in each bounce's nearest-hit
 * pass (the queue balance across networks).  For NET these counts give the network work of
 * a frame: every queried ray is one query, every hit one input gradient (the normal), every
 * shadow ray one query.  stats holds 4 x bounces values (MESH, NET) or (2 + n_nets) x bounces
 * (MULTI). */
ddf_status ddf_render_wavefront(const ddf_scene *scene, const ddf_render_params *p, float *radiance,
                                float *depth, float *normal, uint32_t *stats, void *ws, size_t ws_bytes,
                                ddf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* DDF_H */
