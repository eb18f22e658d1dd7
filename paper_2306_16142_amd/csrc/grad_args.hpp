// Arguments of the network gradient / query sweep (grad.hip), shared by its callers.
#pragma once
#include <cstdint>

#include "common.hpp"
#include "loss_device.hpp"

namespace ddf {

constexpr int kMaxNets = 8;   // networks of one width in a single multi-network launch

struct GradArgs {
    const uint8_t *blob;         // single network: packed blob (ignored when n_nets > 0)
    int depth;                   // single network: depth; multi: the largest depth of the group
    const float *rays;           // [5][n]
    int64_t n;                   // row length of every [k][n] array
    int64_t ray_stride;          // training sweep only: row length of `rays` when it is a column
                                 // range of a longer batch (0: n)
    const int *count_dev;        // single network: only the first *count_dev rays (NULL: all n)
    const float *g_logit_in;     // seeds (NULL = 0)
    const float *g_dist_in;
    const float *t_label;        // training: label distance, +inf = miss (NULL: seeds from g_*_in)
    const float *loss_scalars;   // training: {1 / N, 1 / n_hit}
    LossSpec loss;               // training: which loss forms the seeds (zero: BCE + L1)
    int64_t eik_n;               // training sweep only, > 0: directed Eikonal pairs of eik_n rays
                                 // (64-column tiles: 32 rays, then the same rays moved by eik_h
                                 // along their directions; t_label indexed by ray); the seeds add
                                 // the penalty eik_lam / N sum ((d(x + h d) - d(x)) / h + 1)^2
    float eik_h, eik_lam;
    float *logit_out;            // optional
    float *dist_out;             // optional
    float *g_rays;               // optional [5][n]
    float *ws_gamma;             // side outputs: [65][n] features
    float *ws_h;                 // side outputs: [depth][W][n] hidden activations
    float *ws_delta;             // side outputs: [depth][W][n] adjoints, then [2][n] head seeds
    float *loss_partial;         // training: [gridDim.x]
    bool forward_only;           // stop after logit / distance
    bool grad_hits_only;         // input gradients only where logit > 0 (a hit); other rays of a
                                 // 32-ray block without any hit get no gradient written (streamed
                                 // kernel; the renderer's normals need hits only)
    // several networks of one width in one persistent launch: network k owns the rows
    // [seg_offset[k], seg_offset[k] + seg_count[k]) (device arrays)
    int n_nets;
    const uint8_t *blobs[kMaxNets];
    int depths[kMaxNets];
    const int *seg_offset;
    const int *seg_count;
};

ddf_status grad_dispatch(const ddf_net *net, const GradArgs &args, bool train, hipStream_t s);
// Multi-network launch: every network of the group has `width` and `precision`.
ddf_status grad_dispatch_multi(int width, int precision, const GradArgs &args, hipStream_t s);
int64_t grad_grid(int width, int precision, int64_t n);

// bf16 query / input gradient with the weights streamed through LDS (stream.hip): any depth
// up to 8 at width 128 or 256; args.depth is the largest depth of the launch, and
// args.forward_only selects the query alone.  LDS bytes it needs:
size_t stream_lds_bytes(int width, int depth, int n_nets, bool grad);
ddf_status stream_dispatch(int width, const GradArgs &args, hipStream_t s);

// float32 training sweep with the layer values of 64 rays in LDS (sweep.hip): one network,
// parameter-gradient side outputs only (no input gradient); its grid (one loss partial per
// workgroup) for n rays:
int64_t sweep_grid(int width, int64_t n);
ddf_status sweep_dispatch(int width, const GradArgs &args, hipStream_t s);

// Weight gradient of one affine layer (train.hip): out [M][N] = sum over the n rays of
// A[m][ray] B[k][ray], then out [M][N .. N + M) = sum of A's rows (the bias gradient); rows of A
// and B are contiguous over rays.  The rays are split into fixed chunks whose partial products
// (part: dw_partial_floats(M, N, n) floats; dbpart: as many chunks x M) are added in a fixed
// order, so the result is bitwise reproducible.  accumulate: add to out.
size_t dw_partial_floats(int M, int N, int64_t n);
int dw_chunk(int M, int N);
ddf_status dw_product(const float *A, const float *B, int M, int N, int64_t n, float *part, float *dbpart, float *out,
                      bool accumulate, hipStream_t s);

}  // namespace ddf
