// Training of the network on labelled rays: loss seeds, parameter gradients and Adam.
//
// The paper fits MLP_w to ground-truth field values with Adam (Sec. V-A); the labels here
// come from the triangle labeller (hit flag + distance), the loss is binary cross-entropy
// on the hit logit plus L1 on the distance over hit rays.  One step:
//   1. hit count of the batch -> {1/N, 1/n_hit} on the device (no host round trip);
//   2. the gradient kernel (grad.hip) recomputes the forward pass, seeds the adjoint from
//      the loss and writes the features, hidden activations and adjoints;
//   3. per affine layer, dW = sum over rays of adjoint x input (an MFMA product whose
//      contraction runs over the batch, split into chunks) and db = sum of adjoints; the
//      chunk partials are summed in a fixed order (bitwise reproducible);
//   4. Adam updates the float32 parameters and the packed network is rebuilt.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "mlp_device.hpp"
#include "mlp_layout.hpp"
#include "grad_args.hpp"
#include "rays_device.hpp"

namespace ddf {



namespace {

constexpr int kChunk = 1024;      // rays per split of the batch contraction

// ------------------------------------------------------------------------------ scalars
// Hit count of the labels in two kernels: per-block counts, then one block sums them
// (integer sums: any order gives the same result) and writes {1/N, 1/max(1, hits)}.
constexpr int kCountBlocks = 1024;

__global__ void hit_count_kernel(const float *__restrict__ t_label, int64_t n, unsigned int *part) {
    __shared__ unsigned int red[256];
    unsigned int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += t_label[i] < INFINITY ? 1u : 0u;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void loss_scalars_kernel(const unsigned int *__restrict__ part, int nparts, int64_t n, float *scalars,
                                    unsigned int *count) {
    __shared__ unsigned int red[256];
    unsigned int c = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) c += part[i];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *count = red[0];
        scalars[0] = 1.0f / (float)n;
        scalars[1] = 1.0f / (float)(red[0] > 0 ? red[0] : 1u);
    }
}

// Launches both; `part` holds kCountBlocks counts (it is overwritten later in the stream).
void launch_loss_scalars(const float *t_label, int64_t n, unsigned int *part, float *scalars, unsigned int *count,
                         hipStream_t s) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 2047) / 2048, kCountBlocks));
    hipLaunchKernelGGL(hit_count_kernel, dim3(blocks), dim3(256), 0, s, t_label, n, part);
    hipLaunchKernelGGL(loss_scalars_kernel, dim3(1), dim3(256), 0, s, part, blocks, n, scalars, count);
}

__global__ void sum_partials_kernel(const float *__restrict__ part, int64_t cnt, float *out, bool accumulate) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = accumulate ? *out + red[0] : red[0];
}

// ------------------------------------------------------------------------------ dW = A B^T
// A: [M][n] adjoints, B: [N][n] layer inputs (rows contiguous over rays).  One workgroup
// per (128 x 128 output tile, chunk of kChunk rays).  Stages of 32 rays of both operands
// go through LDS (coalesced 16-byte global loads, rows padded to 36 floats so that the
// MFMA operand reads are free of bank conflicts), double-buffered; eight waves each own a
// 32 x 64 sub-tile (1 x 2 blocks of v_mfma_f32_32x32x2f32), two waves per SIMD.  Lane half
// h contracts rays 16 h .. 16 h + 15 of a stage (the contraction order only pairs A and B of
// the same ray).  The bias gradient is summed by the first 256 threads (two per row).
// part[s][M][N] and dbpart[s][M] receive the chunk's sums.
constexpr int kDwTile = 128;
constexpr int kDwStep = 32;
constexpr int kDwPad = 36;

template <bool kVec4>
__global__ __launch_bounds__(512) void dw_kernel(const float *__restrict__ A, const float *__restrict__ B, int M,
                                                 int N, int64_t n, int splits, int chunk, float *__restrict__ part,
                                                 float *__restrict__ dbpart) {
    __shared__ __attribute__((aligned(16))) float sA[2][kDwTile][kDwPad];
    __shared__ __attribute__((aligned(16))) float sB[2][kDwTile][kDwPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, c = lane & 31;
    const int ntn = (N + kDwTile - 1) / kDwTile;
    const int s = blockIdx.x % splits, tile = blockIdx.x / splits;
    const int m0 = (tile / ntn) * kDwTile, n0 = (tile % ntn) * kDwTile;
    const int64_t k0 = (int64_t)s * chunk;
    const int klen = (int)min<int64_t>(chunk, n - k0);
    const int nstep = (klen + kDwStep - 1) / kDwStep;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
    // global -> register staging: 128 rows x 32 rays per operand = 1024 float4, 2 per thread
    f32x4 ra[2], rb[2];
    auto fetch = [&](int st) {
        const int kb = st * kDwStep;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int idx = tid + 512 * r, row = idx >> 3, k4 = (idx & 7) * 4;
            const int ma = m0 + row, nb = n0 + row;
            const int kk = kb + k4;
            f32x4 va{0.f, 0.f, 0.f, 0.f}, vb{0.f, 0.f, 0.f, 0.f};
            if constexpr (kVec4) {
                if (kk < klen) {   // klen is a multiple of 4 here
                    if (ma < M) va = *reinterpret_cast<const f32x4 *>(A + (int64_t)ma * n + k0 + kk);
                    if (nb < N) vb = *reinterpret_cast<const f32x4 *>(B + (int64_t)nb * n + k0 + kk);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (kk + e < klen) {
                        if (ma < M) va[e] = A[(int64_t)ma * n + k0 + kk + e];
                        if (nb < N) vb[e] = B[(int64_t)nb * n + k0 + kk + e];
                    }
            }
            ra[r] = va;
            rb[r] = vb;
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int idx = tid + 512 * r, row = idx >> 3, k4 = (idx & 7) * 4;
            *reinterpret_cast<f32x4 *>(&sA[buf][row][k4]) = ra[r];
            *reinterpret_cast<f32x4 *>(&sB[buf][row][k4]) = rb[r];
        }
    };
    f32x16 acc[1][2];
#pragma unroll
    for (int i = 0; i < 1; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};
    float dbs = 0.f;   // bias gradient: thread t sums half a row (row t / 2) of the A tile
    fetch(0);
    commit(0);
    __syncthreads();
    for (int st = 0; st < nstep; ++st) {
        const int buf = st & 1;
        if (st + 1 < nstep) fetch(st + 1);
        // a wave whose rows or columns all lie beyond M or N (the head's 2 rows) has no work
        const bool busy = m0 + wm < M && n0 + wn < N;   // wave-uniform
#pragma unroll
        for (int q = 0; q < 4; ++q) {   // four rays per lane half at a time
            if (!busy) break;
            f32x4 a4[1], b4[2];
            a4[0] = *reinterpret_cast<const f32x4 *>(&sA[buf][wm + c][16 * h + 4 * q]);
#pragma unroll
            for (int i = 0; i < 2; ++i) b4[i] = *reinterpret_cast<const f32x4 *>(&sB[buf][wn + 32 * i + c][16 * h + 4 * q]);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < 1; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[i][e], b4[j][e], acc[i][j], 0, 0, 0);
        }
        if (n0 == 0 && tid < 256) {
            const f32x4 *row = reinterpret_cast<const f32x4 *>(&sA[buf][tid >> 1][16 * (tid & 1)]);
#pragma unroll
            for (int e = 0; e < 4; ++e) dbs += (row[e][0] + row[e][1]) + (row[e][2] + row[e][3]);
        }
        if (st + 1 < nstep) commit(buf ^ 1);
        __syncthreads();
    }
    float *dst = part + (int64_t)s * M * N;
#pragma unroll
    for (int i = 0; i < 1; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int m = m0 + wm + 32 * i + 8 * (q / 4) + 4 * h + (q % 4);
                const int k = n0 + wn + 32 * j + c;
                if (m < M && k < N) dst[(int64_t)m * N + k] = acc[i][j][q];
            }
    if (n0 == 0 && tid < 256) {
        const float t = dbs + __shfl_xor(dbs, 1);
        const int m = m0 + (tid >> 1);
        if ((tid & 1) == 0 && m < M) dbpart[(int64_t)s * M + m] = t;
    }
}

// g[W block] (+)= sum_s part[s], g[b block] (+)= sum_s dbpart[s]  (fixed summation order).
// Four lanes share an element: lane q sums the splits q, q + 4, q + 8, ... and lane 0 of the
// group adds the four sums in lane order, so more loads are in flight per element.
constexpr int kReduceLanes = 4;   // the shuffles below take four partial sums
__global__ void reduce_dw_kernel(const float *__restrict__ part, const float *__restrict__ dbpart, int M, int N,
                                 int splits, float *__restrict__ g, bool accumulate) {
    const int64_t total = (int64_t)M * N + M;
    const int q = threadIdx.x % kReduceLanes;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kReduceLanes);
    // every lane runs the same number of iterations (the shuffles need the whole wave)
    for (int64_t e0 = (int64_t)blockIdx.x * (blockDim.x / kReduceLanes); e0 < total; e0 += stride) {
        const int64_t e = e0 + threadIdx.x / kReduceLanes;
        float s = 0.f;
        if (e < (int64_t)M * N) {
            for (int k = q; k < splits; k += kReduceLanes) s += part[(int64_t)k * M * N + e];
        } else if (e < total) {
            const int64_t m = e - (int64_t)M * N;
            for (int k = q; k < splits; k += kReduceLanes) s += dbpart[(int64_t)k * M + m];
        }
        const int lead = (threadIdx.x & 63) & ~(kReduceLanes - 1);
        const float s0 = __shfl(s, lead), s1 = __shfl(s, lead + 1), s2 = __shfl(s, lead + 2), s3 = __shfl(s, lead + 3);
        if (q == 0 && e < total) {
            const float t = ((s0 + s1) + s2) + s3;
            g[e] = accumulate ? g[e] + t : t;
        }
    }
}

// ------------------------------------------------------------------------------ Adam
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t count, float lr, float beta1, float beta2, float eps,
                            float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = beta1 * m[i] + (1.f - beta1) * gi;
        const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// ------------------------------------------------------------------------------ loss seeds
__global__ void loss_seeds_kernel(const float *__restrict__ logit, const float *__restrict__ dist,
                                  const float *__restrict__ t_label, int64_t n, const float *__restrict__ scalars,
                                  LossSpec ls, float *__restrict__ g_logit, float *__restrict__ g_dist,
                                  float *__restrict__ part) {
    __shared__ float red[256];
    const float inv_n = scalars[0], inv_nhit = scalars[1];
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float gl, gd;
        acc += ray_loss(logit[i], dist[i], t_label[i], inv_n, inv_nhit, ls, gl, gd);
        g_logit[i] = gl;
        g_dist[i] = gd;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

// Rays per split of the batch contraction for an M x N product: layers of fewer than four
// 128 x 128 output tiles split the rays twice as finely, so that they still occupy every CU.
int dw_chunk(int M, int N) {
    const int tiles = ((M + kDwTile - 1) / kDwTile) * ((N + kDwTile - 1) / kDwTile);
    return tiles >= 4 ? kChunk : kChunk / 2;
}

size_t dw_partial_floats(int M, int N, int64_t n) {
    return (size_t)((n + dw_chunk(M, N) - 1) / dw_chunk(M, N)) * M * N;
}

ddf_status dw_product(const float *A, const float *B, int M, int N, int64_t n, float *part, float *dbpart, float *out,
                      bool accumulate, hipStream_t s) {
    const int tiles = ((M + kDwTile - 1) / kDwTile) * ((N + kDwTile - 1) / kDwTile);
    const int chunk = dw_chunk(M, N);
    const int splits = (int)((n + chunk - 1) / chunk);
    const unsigned blocks = (unsigned)(tiles * splits);
    if (n % 4 == 0)
        hipLaunchKernelGGL(dw_kernel<true>, dim3(blocks), dim3(512), 0, s, A, B, M, N, n, splits, chunk, part, dbpart);
    else
        hipLaunchKernelGGL(dw_kernel<false>, dim3(blocks), dim3(512), 0, s, A, B, M, N, n, splits, chunk, part, dbpart);
    if (ddf_status st = launch_status("ddf parameter gradient")) return st;
    const int64_t total = (int64_t)M * N + M;
    hipLaunchKernelGGL(reduce_dw_kernel, dim3((unsigned)std::min<int64_t>((total + 63) / 64, 4096)), dim3(256), 0, s,
                       part, dbpart, M, N, splits, out, accumulate);
    return launch_status("ddf parameter gradient reduction");
}

namespace {

// ------------------------------------------------------------------------------ workspace
struct TrainWs {
    float *gamma, *h, *delta, *loss_part, *scalars, *part, *dbpart;
    unsigned int *count;
    size_t bytes;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

TrainWs train_ws(int width, int depth, int64_t n, void *base) {
    TrainWs w{};
    uint8_t *p = reinterpret_cast<uint8_t *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        uint8_t *q = p ? p + off : nullptr;
        off += align256(bytes);
        return q;
    };
    const int64_t splits = (n + kChunk - 1) / kChunk;
    const int maxN = std::max(width, kInDim);
    w.gamma = reinterpret_cast<float *>(take((size_t)kInDim * n * 4));
    w.h = reinterpret_cast<float *>(take((size_t)depth * width * n * 4));
    w.delta = reinterpret_cast<float *>(take(((size_t)depth * width + 2) * n * 4));
    w.loss_part = reinterpret_cast<float *>(take(4096 * 4));
    w.scalars = reinterpret_cast<float *>(take(16));
    w.count = reinterpret_cast<unsigned int *>(take(16));
    // partials for up to twice the splits (layers of few output tiles use half-size chunks)
    w.part = reinterpret_cast<float *>(take((size_t)2 * splits * width * maxN * 4));
    w.dbpart = reinterpret_cast<float *>(take((size_t)2 * splits * width * 4));
    w.bytes = off;
    return w;
}

// Parameter gradients of all layers from the stored features / activations / adjoints.
ddf_status param_grads(int width, int depth, int64_t n, const TrainWs &w, float *g_params, bool accumulate,
                       hipStream_t s) {
    int64_t off = 0;
    for (int l = 0; l <= depth; ++l) {
        const int M = l == depth ? 2 : width;
        const int N = l == 0 ? kInDim : width;
        const float *A = l == depth ? w.delta + (int64_t)depth * width * n : w.delta + (int64_t)l * width * n;
        const float *B = l == 0 ? w.gamma : w.h + (int64_t)(l - 1) * width * n;
        if (ddf_status st = dw_product(A, B, M, N, n, w.part, w.dbpart, g_params + off, accumulate, s)) return st;
        off += (int64_t)M * N + M;
    }
    return DDF_OK;
}

ddf_status check_net(const ddf_net *net, const char *who, bool fp32_only) {
    DDF_REQUIRE(net && net->packed, DDF_ERR_INVALID_ARG, "%s: NULL network", who);
    DDF_REQUIRE(net->width == 128 || net->width == 256, DDF_ERR_UNSUPPORTED, "%s: width %d not supported", who, net->width);
    DDF_REQUIRE(net->depth >= 1 && net->depth <= 8, DDF_ERR_UNSUPPORTED, "%s: depth %d not supported", who, net->depth);
    if (fp32_only)
        DDF_REQUIRE(net->precision == kFP32, DDF_ERR_UNSUPPORTED, "%s: parameter gradients need a float32 network", who);
    else
        DDF_REQUIRE(net->precision == kFP32 || net->precision == kBF16, DDF_ERR_UNSUPPORTED,
                    "%s: input gradients need a float32 or bfloat16 network", who);
    return DDF_OK;
}

}  // namespace
}  // namespace ddf

using namespace ddf;

extern "C" ddf_status ddf_train_workspace_size(int32_t width, int32_t depth, int64_t n, size_t *bytes) {
    DDF_REQUIRE(bytes && n >= 0 && width > 0 && depth > 0, DDF_ERR_INVALID_ARG, "ddf_train_workspace_size: bad argument");
    *bytes = train_ws(width, depth, n, nullptr).bytes;
    return DDF_OK;
}

extern "C" ddf_status ddf_backward(const ddf_net *net, const float *rays, int64_t n, const float *g_logit,
                                   const float *g_dist, float *g_rays, float *g_params, uint32_t flags, void *ws,
                                   size_t ws_bytes, ddf_stream stream) {
    if (ddf_status st = check_net(net, "ddf_backward", g_params != nullptr)) return st;
    DDF_REQUIRE(n >= 0, DDF_ERR_INVALID_ARG, "ddf_backward: negative n");
    DDF_REQUIRE((flags & ~1u) == 0, DDF_ERR_INVALID_ARG, "ddf_backward: unknown flags 0x%x", flags);
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(rays, DDF_ERR_INVALID_ARG, "ddf_backward: NULL rays");
    DDF_REQUIRE(g_rays || g_params, DDF_ERR_INVALID_ARG, "ddf_backward: nothing to compute");
    hipStream_t s = as_stream(stream);
    GradArgs a{};
    a.blob = (const uint8_t *)net->packed;
    a.depth = net->depth;
    a.rays = rays;
    a.n = n;
    a.g_logit_in = g_logit;
    a.g_dist_in = g_dist;
    a.g_rays = g_rays;
    if (!g_params) return grad_dispatch(net, a, false, s);
    const TrainWs need = train_ws(net->width, net->depth, n, nullptr);
    DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE, "ddf_backward: workspace of %zu bytes needed",
                need.bytes);
    const TrainWs w = train_ws(net->width, net->depth, n, ws);
    DDF_REQUIRE(grad_grid(net->width, net->precision, n) <= 4096, DDF_ERR_UNSUPPORTED, "ddf_backward: grid too large");
    a.ws_gamma = w.gamma;
    a.ws_h = w.h;
    a.ws_delta = w.delta;
    a.loss_partial = w.loss_part;
    if (ddf_status st = grad_dispatch(net, a, true, s)) return st;
    return param_grads(net->width, net->depth, n, w, g_params, (flags & 1u) != 0, s);
}

namespace ddf {
namespace {
ddf_status check_loss(const ddf_loss *loss, LossSpec *out, const char *who) {
    if (!loss) {
        *out = LossSpec{0, 0.f};
        return DDF_OK;
    }
    DDF_REQUIRE(loss->kind >= DDF_LOSS_BCE_L1 && loss->kind <= DDF_LOSS_SQUISH, DDF_ERR_INVALID_ARG,
                "%s: unknown loss kind %d", who, loss->kind);
    DDF_REQUIRE(loss->kind != DDF_LOSS_CLAMP || (std::isfinite(loss->delta) && loss->delta > 0.f), DDF_ERR_INVALID_ARG,
                "%s: the clamp loss needs a finite delta > 0", who);
    *out = LossSpec{loss->kind, loss->delta};
    return DDF_OK;
}
}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_loss_seeds_ex(const float *logit, const float *dist, const float *t_label, int64_t n,
                                        const ddf_loss *loss, float *g_logit, float *g_dist, float *loss_out, void *ws,
                                        size_t ws_bytes, ddf_stream stream) {
    LossSpec ls;
    if (ddf_status st = check_loss(loss, &ls, "ddf_loss_seeds")) return st;
    DDF_REQUIRE(n > 0 && logit && dist && t_label && g_logit && g_dist && loss_out, DDF_ERR_INVALID_ARG,
                "ddf_loss_seeds: bad argument");
    DDF_REQUIRE(ws && ws_bytes >= 1024 * 4 + 64, DDF_ERR_WORKSPACE, "ddf_loss_seeds: workspace of %d bytes needed",
                1024 * 4 + 64);
    hipStream_t s = as_stream(stream);
    float *part = reinterpret_cast<float *>(ws);
    float *scalars = part + 1024;
    unsigned int *count = reinterpret_cast<unsigned int *>(scalars + 4);
    launch_loss_scalars(t_label, n, reinterpret_cast<unsigned int *>(part), scalars, count, s);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(loss_seeds_kernel, dim3(blocks), dim3(256), 0, s, logit, dist, t_label, n, scalars, ls, g_logit,
                       g_dist, part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)blocks, loss_out, false);
    return launch_status("ddf_loss_seeds");
}

extern "C" ddf_status ddf_loss_seeds(const float *logit, const float *dist, const float *t_label, int64_t n,
                                     float *g_logit, float *g_dist, float *loss_out, void *ws, size_t ws_bytes,
                                     ddf_stream stream) {
    return ddf_loss_seeds_ex(logit, dist, t_label, n, nullptr, g_logit, g_dist, loss_out, ws, ws_bytes, stream);
}

extern "C" ddf_status ddf_adam_step(float *params, const float *grads, float *m, float *v, int64_t count, int64_t step,
                                    float lr, float beta1, float beta2, float eps, ddf_stream stream) {
    DDF_REQUIRE(params && grads && m && v && count > 0 && step >= 1, DDF_ERR_INVALID_ARG, "ddf_adam_step: bad argument");
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)std::min<int64_t>((count + 255) / 256, 4096)), dim3(256), 0,
                       as_stream(stream), params, grads, m, v, count, lr, beta1, beta2, eps, bc1, bc2);
    return launch_status("ddf_adam_step");
}

extern "C" ddf_status ddf_pack_net(const float *params, int32_t width, int32_t depth, int32_t precision,
                                   const float *scales, void *packed, ddf_stream stream);

namespace ddf {
namespace {
// Adam on the flat parameters (float32 layers of the network) and repacking of `net`.
ddf_status adam_and_repack(const ddf_net *net, float *params, float *adam_m, float *adam_v, const float *g_params,
                           int64_t step, float lr, ddf_stream stream) {
    int64_t count = 0;
    int in = kInDim;
    for (int l = 0; l <= net->depth; ++l) {
        const int out = l == net->depth ? 2 : net->width;
        count += (int64_t)out * in + out;
        in = net->width;
    }
    if (ddf_status st = ddf_adam_step(params, g_params, adam_m, adam_v, count, step, lr, 0.9f, 0.999f, 1e-8f, stream))
        return st;
    return ddf_pack_net(params, net->width, net->depth, net->precision, nullptr, const_cast<void *>(net->packed), stream);
}
}  // namespace
}  // namespace ddf

namespace ddf {
namespace {
ddf_status train_step_whole(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step, float lr,
                            const float *rays, const float *t_label, int64_t n, LossSpec ls, float *loss_out,
                            float *g_params, void *ws, size_t ws_bytes, ddf_stream stream) {
    if (ddf_status st = check_net(net, "ddf_train_step", true)) return st;
    DDF_REQUIRE(params && adam_m && adam_v && rays && t_label && loss_out && g_params && n > 0 && step >= 1,
                DDF_ERR_INVALID_ARG, "ddf_train_step: bad argument");
    const TrainWs need = train_ws(net->width, net->depth, n, nullptr);
    DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE, "ddf_train_step: workspace of %zu bytes needed",
                need.bytes);
    const int64_t grid = grad_grid(net->width, net->precision, n);
    DDF_REQUIRE(grid <= 4096, DDF_ERR_UNSUPPORTED, "ddf_train_step: grid too large");
    hipStream_t s = as_stream(stream);
    const TrainWs w = train_ws(net->width, net->depth, n, ws);
    launch_loss_scalars(t_label, n, reinterpret_cast<unsigned int *>(w.loss_part), w.scalars, w.count, s);
    if (ddf_status st = launch_status("ddf_train_step")) return st;
    GradArgs a{};
    a.blob = (const uint8_t *)net->packed;
    a.depth = net->depth;
    a.rays = rays;
    a.n = n;
    a.t_label = t_label;
    a.loss_scalars = w.scalars;
    a.loss = ls;
    a.ws_gamma = w.gamma;
    a.ws_h = w.h;
    a.ws_delta = w.delta;
    a.loss_partial = w.loss_part;
    if (ddf_status st = grad_dispatch(net, a, true, s)) return st;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, w.loss_part, grid, loss_out, false);
    if (ddf_status st = param_grads(net->width, net->depth, n, w, g_params, false, s)) return st;
    return adam_and_repack(net, params, adam_m, adam_v, g_params, step, lr, stream);
}
}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_train_step(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step,
                                     float lr, const float *rays, const float *t_label, int64_t n, float *loss_out,
                                     float *g_params, void *ws, size_t ws_bytes, ddf_stream stream) {
    return train_step_whole(net, params, adam_m, adam_v, step, lr, rays, t_label, n, LossSpec{0, 0.f}, loss_out,
                            g_params, ws, ws_bytes, stream);
}

namespace ddf {
namespace {
ddf_status train_step_chunks(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step, float lr,
                             const float *rays, const float *t_label, int64_t n, int64_t chunk, LossSpec ls,
                             float *loss_out, float *g_params, void *ws, size_t ws_bytes, ddf_stream stream) {
    if (ddf_status st = check_net(net, "ddf_train_step_chunked", true)) return st;
    DDF_REQUIRE(params && adam_m && adam_v && rays && t_label && loss_out && g_params && n > 0 && chunk > 0 &&
                    step >= 1,
                DDF_ERR_INVALID_ARG, "ddf_train_step_chunked: bad argument");
    chunk = std::min(chunk, n);
    const TrainWs need = train_ws(net->width, net->depth, chunk, nullptr);
    DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE,
                "ddf_train_step_chunked: workspace of %zu bytes needed", need.bytes);
    DDF_REQUIRE(grad_grid(net->width, net->precision, chunk) <= 4096, DDF_ERR_UNSUPPORTED,
                "ddf_train_step_chunked: grid too large");
    hipStream_t s = as_stream(stream);
    const TrainWs w = train_ws(net->width, net->depth, chunk, ws);
    // the loss normalisation (1 / N, 1 / hits) of the whole batch, then every chunk's sweep
    // (its forward pass recomputed, its activations only in the chunk workspace) adds its
    // loss and parameter gradient in chunk order
    launch_loss_scalars(t_label, n, reinterpret_cast<unsigned int *>(w.loss_part), w.scalars, w.count, s);
    if (ddf_status st = launch_status("ddf_train_step_chunked")) return st;
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
        const int64_t m = std::min(chunk, n - c0);
        GradArgs a{};
        a.blob = (const uint8_t *)net->packed;
        a.depth = net->depth;
        a.rays = rays + c0;
        a.ray_stride = n;
        a.n = m;
        a.t_label = t_label + c0;
        a.loss_scalars = w.scalars;
        a.loss = ls;
        a.ws_gamma = w.gamma;
        a.ws_h = w.h;
        a.ws_delta = w.delta;
        a.loss_partial = w.loss_part;
        if (ddf_status st = sweep_dispatch(net->width, a, s)) return st;
        hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, w.loss_part,
                           grad_grid(net->width, net->precision, m), loss_out, c0 > 0);
        if (ddf_status st = param_grads(net->width, net->depth, m, w, g_params, c0 > 0, s)) return st;
    }
    return adam_and_repack(net, params, adam_m, adam_v, g_params, step, lr, stream);
}
}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_train_step_chunked(const ddf_net *net, float *params, float *adam_m, float *adam_v,
                                             int64_t step, float lr, const float *rays, const float *t_label,
                                             int64_t n, int64_t chunk, float *loss_out, float *g_params, void *ws,
                                             size_t ws_bytes, ddf_stream stream) {
    return train_step_chunks(net, params, adam_m, adam_v, step, lr, rays, t_label, n, chunk, LossSpec{0, 0.f}, loss_out,
                             g_params, ws, ws_bytes, stream);
}

extern "C" ddf_status ddf_train_step_ex(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step,
                                        float lr, const float *rays, const float *t_label, int64_t n, int64_t chunk,
                                        const ddf_loss *loss, float *loss_out, float *g_params, void *ws,
                                        size_t ws_bytes, ddf_stream stream) {
    LossSpec ls;
    if (ddf_status st = check_loss(loss, &ls, "ddf_train_step_ex")) return st;
    DDF_REQUIRE(chunk >= 0, DDF_ERR_INVALID_ARG, "ddf_train_step_ex: negative chunk");
    if (chunk == 0)
        return train_step_whole(net, params, adam_m, adam_v, step, lr, rays, t_label, n, ls, loss_out, g_params, ws,
                                ws_bytes, stream);
    return train_step_chunks(net, params, adam_m, adam_v, step, lr, rays, t_label, n, chunk, ls, loss_out, g_params,
                             ws, ws_bytes, stream);
}

// ------------------------------------------------------------------------------ directed Eikonal
// Training with the directed Eikonal penalty of Eq. 2 (Sec. III-A): along its own ray the
// field falls at unit rate.  The derivative along the ray is taken as a forward difference,
// r = (phi(x + h d) - phi(x)) / h + 1, so the step needs first-order gradients only: the batch
// is doubled (rays at x and at x + h d), both halves go through the network, the seeds are the
// chosen loss's on the first half plus the penalty's on both, and one backward sweep over the
// doubled batch gives the parameter gradient.
namespace ddf {
namespace {

// rays [5][2n]: columns 0..n-1 at the origins, n..2n-1 moved by h along the unit direction.
// Directed Eikonal pairs in the training sweep's 64-column tiles: tile j holds rays 32 j ..
// 32 j + 31 (columns 64 j + c), then the same rays moved by h along their unit directions
// (columns 64 j + 32 + c); columns past the n rays are zero rays (their seeds are zero).
__global__ void eikonal_pairs_kernel(const float *__restrict__ orig, const float *__restrict__ dir, int64_t n,
                                     int64_t m, float h, float *__restrict__ rays) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // ray slot, < m / 2
    if (2 * i >= m) return;
    const int64_t ca = (i / 32) * 64 + i % 32, cb = ca + 32;
    if (i >= n) {
#pragma unroll
        for (int c = 0; c < 5; ++c) rays[c * m + ca] = rays[c * m + cb] = 0.f;
        return;
    }
    const float dx = dir[i], dy = dir[n + i], dz = dir[2 * n + i];
    float theta, phi;
    dir_angles(dx, dy, dz, theta, phi);
    const float inv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
    const float d[3] = {dx * inv, dy * inv, dz * inv};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float o = orig[c * n + i];
        rays[c * m + ca] = o;
        rays[c * m + cb] = fmaf(h, d[c], o);
    }
    rays[3 * m + ca] = rays[3 * m + cb] = theta;
    rays[4 * m + ca] = rays[4 * m + cb] = phi;
}

// Columns of the paired batch of n rays: 64 per 32 rays (the last tile padded).
inline int64_t eik_cols(int64_t n) { return (n + 31) / 32 * 64; }

// Workspace: the paired rays [5][cols] | the training sweep's workspace for cols columns.
struct EikWs {
    float *rays;
    TrainWs tw;
    size_t bytes;
};

EikWs eik_ws(int width, int depth, int64_t n, void *base) {
    EikWs w{};
    const int64_t m = eik_cols(n);
    const size_t rb = align256((size_t)5 * m * 4);
    w.rays = base ? (float *)base : nullptr;
    w.tw = train_ws(width, depth, m, base ? (uint8_t *)base + rb : nullptr);
    w.bytes = rb + w.tw.bytes;
    return w;
}

}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_eikonal_workspace_size(int32_t width, int32_t depth, int64_t n, size_t *bytes) {
    DDF_REQUIRE(bytes && n >= 0, DDF_ERR_INVALID_ARG, "ddf_eikonal_workspace_size: bad argument");
    *bytes = eik_ws(width, depth, n, nullptr).bytes;
    return DDF_OK;
}

extern "C" ddf_status ddf_train_step_eikonal(const ddf_net *net, float *params, float *adam_m, float *adam_v,
                                             int64_t step, float lr, const float *orig, const float *dir,
                                             const float *t_label, int64_t n, float h, float lambda,
                                             const ddf_loss *loss, float *loss_out, float *g_params, void *ws,
                                             size_t ws_bytes, ddf_stream stream) {
    if (ddf_status st = check_net(net, "ddf_train_step_eikonal", true)) return st;
    LossSpec ls;
    if (ddf_status st = check_loss(loss, &ls, "ddf_train_step_eikonal")) return st;
    DDF_REQUIRE(params && adam_m && adam_v && orig && dir && t_label && loss_out && g_params && n > 0 && step >= 1,
                DDF_ERR_INVALID_ARG, "ddf_train_step_eikonal: bad argument");
    DDF_REQUIRE(std::isfinite(h) && h > 0.f && std::isfinite(lambda) && lambda >= 0.f, DDF_ERR_INVALID_ARG,
                "ddf_train_step_eikonal: need a finite h > 0 and lambda >= 0");
    const EikWs need = eik_ws(net->width, net->depth, n, nullptr);
    DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE,
                "ddf_train_step_eikonal: workspace of %zu bytes needed", need.bytes);
    const EikWs w = eik_ws(net->width, net->depth, n, ws);
    const int64_t m = eik_cols(n);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(eikonal_pairs_kernel, dim3((unsigned)((m / 2 + 255) / 256)), dim3(256), 0, s, orig, dir, n, m, h,
                       w.rays);
    launch_loss_scalars(t_label, n, reinterpret_cast<unsigned int *>(w.tw.loss_part), w.tw.scalars, w.tw.count, s);
    if (ddf_status st = launch_status("ddf_train_step_eikonal")) return st;
    // one training sweep over the pairs: forward, the loss and penalty seeds of each pair in
    // its workgroup, adjoints; then the weight-gradient products of the m columns
    GradArgs a{};
    a.blob = (const uint8_t *)net->packed;
    a.depth = net->depth;
    a.rays = w.rays;
    a.n = m;
    a.t_label = t_label;
    a.loss_scalars = w.tw.scalars;
    a.loss = ls;
    a.eik_n = n;
    a.eik_h = h;
    a.eik_lam = lambda;
    a.ws_gamma = w.tw.gamma;
    a.ws_h = w.tw.h;
    a.ws_delta = w.tw.delta;
    a.loss_partial = w.tw.loss_part;
    if (ddf_status st = sweep_dispatch(net->width, a, s)) return st;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, w.tw.loss_part, sweep_grid(net->width, m), loss_out,
                       false);
    if (ddf_status st = param_grads(net->width, net->depth, m, w.tw, g_params, false, s)) return st;
    return adam_and_repack(net, params, adam_m, adam_v, g_params, step, lr, stream);
}
