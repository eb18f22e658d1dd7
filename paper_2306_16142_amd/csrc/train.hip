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

namespace ddf {



namespace {

constexpr int kChunk = 2048;      // rays per split of the batch contraction
constexpr int kGemmTile = 64;     // output tile per wave (2 x 2 MFMA blocks)

// ------------------------------------------------------------------------------ scalars
__global__ void loss_scalars_kernel(const float *__restrict__ t_label, int64_t n, float *scalars,
                                    unsigned int *count) {
    // single block: count hits (t < +inf) in a fixed order, then write {1/N, 1/max(1, hits)}
    __shared__ unsigned int red[256];
    unsigned int c = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) c += t_label[i] < INFINITY ? 1u : 0u;
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

__global__ void sum_partials_kernel(const float *__restrict__ part, int64_t cnt, float *out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------------------------ dW = A B^T
// A: [M][n] adjoints, B: [N][n] layer inputs (rows contiguous over rays).  One wave per
// (64 x 64 output tile, chunk of kChunk rays); lane half h contracts the first or the
// second half of the chunk (the MFMA's k index pairs the same ray in A and B).
// part[s][M][N] and dbpart[s][M] receive the chunk's sums.
template <bool kVec4>
__global__ __launch_bounds__(256) void dw_kernel(const float *__restrict__ A, const float *__restrict__ B, int M,
                                                 int N, int64_t n, int splits, float *__restrict__ part,
                                                 float *__restrict__ dbpart) {
    const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31;
    const int mt = (M + kGemmTile - 1) / kGemmTile, nt = (N + kGemmTile - 1) / kGemmTile;
    const int64_t job = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (job >= (int64_t)mt * nt * splits) return;
    const int s = (int)(job % splits);
    const int tile = (int)(job / splits);
    const int m0 = (tile / nt) * kGemmTile, n0 = (tile % nt) * kGemmTile;
    // rays of this chunk: lane half 0 takes the first kChunk / 2, half 1 the rest; every
    // loop bound below is the same for the whole wave (MFMAs must not run divergent)
    const int64_t chunk_len = std::min<int64_t>(kChunk, n - (int64_t)s * kChunk);
    const int64_t len0 = std::min<int64_t>(kChunk / 2, chunk_len);
    const int64_t len1 = std::max<int64_t>(0, chunk_len - kChunk / 2);
    const int64_t len = h ? len1 : len0;
    const int64_t r0 = (int64_t)s * kChunk + h * (kChunk / 2);
    const float *arow[2];
    const float *brow[2];
    bool aok[2], bok[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = m0 + 32 * i + c, k = n0 + 32 * i + c;
        aok[i] = m < M;
        bok[i] = k < N;
        arow[i] = A + (int64_t)(aok[i] ? m : 0) * n + r0;
        brow[i] = B + (int64_t)(bok[i] ? k : 0) * n + r0;
    }
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;
    float dbs[2] = {0.f, 0.f};
    int64_t ks = 0;
    if constexpr (kVec4) {
        const int64_t vlen = (len1 / 4) * 4;   // len1 <= len0: both halves have these rays
        for (; ks < vlen; ks += 4) {
            f32x4 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = aok[i] ? *reinterpret_cast<const f32x4 *>(arow[i] + ks) : f32x4{0.f, 0.f, 0.f, 0.f};
                bv[i] = bok[i] ? *reinterpret_cast<const f32x4 *>(brow[i] + ks) : f32x4{0.f, 0.f, 0.f, 0.f};
                dbs[i] += (av[i][0] + av[i][1]) + (av[i][2] + av[i][3]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
        }
    }
    for (; ks < len0; ++ks) {
        float av[2], bv[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            av[i] = (aok[i] && ks < len) ? arow[i][ks] : 0.f;
            bv[i] = (bok[i] && ks < len) ? brow[i][ks] : 0.f;
            dbs[i] += av[i];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    float *dst = part + (int64_t)s * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int m = m0 + 32 * i + 8 * (q / 4) + 4 * h + (q % 4);
                const int k = n0 + 32 * j + c;
                if (m < M && k < N) dst[(int64_t)m * N + k] = acc[i][j][q];
            }
    if (n0 == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float t = dbs[i] + __shfl_xor(dbs[i], 32);
            const int m = m0 + 32 * i + c;
            if (h == 0 && m < M) dbpart[(int64_t)s * M + m] = t;
        }
    }
}

// g[W block] (+)= sum_s part[s], g[b block] (+)= sum_s dbpart[s]  (fixed summation order)
__global__ void reduce_dw_kernel(const float *__restrict__ part, const float *__restrict__ dbpart, int M, int N,
                                 int splits, float *__restrict__ g, bool accumulate) {
    const int64_t total = (int64_t)M * N + M;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        if (e < (int64_t)M * N) {
            for (int k = 0; k < splits; ++k) s += part[(int64_t)k * M * N + e];
        } else {
            const int64_t m = e - (int64_t)M * N;
            for (int k = 0; k < splits; ++k) s += dbpart[(int64_t)k * M + m];
        }
        g[e] = accumulate ? g[e] + s : s;
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
                                  float *__restrict__ g_logit, float *__restrict__ g_dist, float *__restrict__ part) {
    __shared__ float red[256];
    const float inv_n = scalars[0], inv_nhit = scalars[1];
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float z = logit[i], d = dist[i], t = t_label[i];
        const float y = t < INFINITY ? 1.f : 0.f;
        const float diff = d - (y > 0.f ? t : 0.f);
        g_logit[i] = (1.f / (1.f + expf(-z)) - y) * inv_n;
        g_dist[i] = y > 0.f ? (diff > 0.f ? inv_nhit : (diff < 0.f ? -inv_nhit : 0.f)) : 0.f;
        acc += (fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z)))) * inv_n + y * fabsf(diff) * inv_nhit;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

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
    w.part = reinterpret_cast<float *>(take((size_t)splits * width * maxN * 4));
    w.dbpart = reinterpret_cast<float *>(take((size_t)splits * width * 4));
    w.bytes = off;
    return w;
}

// Parameter gradients of all layers from the stored features / activations / adjoints.
ddf_status param_grads(int width, int depth, int64_t n, const TrainWs &w, float *g_params, bool accumulate,
                       hipStream_t s) {
    const int splits = (int)((n + kChunk - 1) / kChunk);
    int64_t off = 0;
    for (int l = 0; l <= depth; ++l) {
        const int M = l == depth ? 2 : width;
        const int N = l == 0 ? kInDim : width;
        const float *A = l == depth ? w.delta + (int64_t)depth * width * n : w.delta + (int64_t)l * width * n;
        const float *B = l == 0 ? w.gamma : w.h + (int64_t)(l - 1) * width * n;
        const int64_t jobs = (int64_t)((M + kGemmTile - 1) / kGemmTile) * ((N + kGemmTile - 1) / kGemmTile) * splits;
        const unsigned blocks = (unsigned)((jobs + 3) / 4);
        if (n % 4 == 0)
            hipLaunchKernelGGL(dw_kernel<true>, dim3(blocks), dim3(256), 0, s, A, B, M, N, n, splits, w.part, w.dbpart);
        else
            hipLaunchKernelGGL(dw_kernel<false>, dim3(blocks), dim3(256), 0, s, A, B, M, N, n, splits, w.part, w.dbpart);
        if (ddf_status st = launch_status("ddf parameter gradient")) return st;
        const int64_t total = (int64_t)M * N + M;
        hipLaunchKernelGGL(reduce_dw_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)), dim3(256), 0, s,
                           w.part, w.dbpart, M, N, splits, g_params + off, accumulate);
        if (ddf_status st = launch_status("ddf parameter gradient reduction")) return st;
        off += total;
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

extern "C" ddf_status ddf_loss_seeds(const float *logit, const float *dist, const float *t_label, int64_t n,
                                     float *g_logit, float *g_dist, float *loss_out, void *ws, size_t ws_bytes,
                                     ddf_stream stream) {
    DDF_REQUIRE(n > 0 && logit && dist && t_label && g_logit && g_dist && loss_out, DDF_ERR_INVALID_ARG,
                "ddf_loss_seeds: bad argument");
    DDF_REQUIRE(ws && ws_bytes >= 1024 * 4 + 64, DDF_ERR_WORKSPACE, "ddf_loss_seeds: workspace of %d bytes needed",
                1024 * 4 + 64);
    hipStream_t s = as_stream(stream);
    float *part = reinterpret_cast<float *>(ws);
    float *scalars = part + 1024;
    unsigned int *count = reinterpret_cast<unsigned int *>(scalars + 4);
    hipLaunchKernelGGL(loss_scalars_kernel, dim3(1), dim3(256), 0, s, t_label, n, scalars, count);
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(loss_seeds_kernel, dim3(blocks), dim3(256), 0, s, logit, dist, t_label, n, scalars, g_logit,
                       g_dist, part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)blocks, loss_out);
    return launch_status("ddf_loss_seeds");
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

extern "C" ddf_status ddf_train_step(const ddf_net *net, float *params, float *adam_m, float *adam_v, int64_t step,
                                     float lr, const float *rays, const float *t_label, int64_t n, float *loss_out,
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
    hipLaunchKernelGGL(loss_scalars_kernel, dim3(1), dim3(256), 0, s, t_label, n, w.scalars, w.count);
    if (ddf_status st = launch_status("ddf_train_step")) return st;
    GradArgs a{};
    a.blob = (const uint8_t *)net->packed;
    a.depth = net->depth;
    a.rays = rays;
    a.n = n;
    a.t_label = t_label;
    a.loss_scalars = w.scalars;
    a.ws_gamma = w.gamma;
    a.ws_h = w.h;
    a.ws_delta = w.delta;
    a.loss_partial = w.loss_part;
    if (ddf_status st = grad_dispatch(net, a, true, s)) return st;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, w.loss_part, grid, loss_out);
    if (ddf_status st = param_grads(net->width, net->depth, n, w, g_params, false, s)) return st;
    int64_t count = 0;
    {
        int in = kInDim;
        for (int l = 0; l <= net->depth; ++l) {
            const int out = l == net->depth ? 2 : net->width;
            count += (int64_t)out * in + out;
            in = net->width;
        }
    }
    if (ddf_status st = ddf_adam_step(params, g_params, adam_m, adam_v, count, step, lr, 0.9f, 0.999f, 1e-8f, stream))
        return st;
    return ddf_pack_net(params, net->width, net->depth, net->precision, nullptr, const_cast<void *>(net->packed), stream);
}
