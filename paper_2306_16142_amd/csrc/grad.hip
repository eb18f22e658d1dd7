// Reverse-mode sweep of the network for whole waves of rays.
//
// The gradient of the field with respect to the query point gives the surface normal
// (Eq. 3, Sec. IV-B: the paper takes it with automatic differentiation; here it is a
// hand-written adjoint).  The same sweep, with the loss gradient as its seed and the
// layer activations and adjoints written out, is the backward half of training.
//
// Per wave of 32 NB rays, in registers: the forward pass is recomputed (its ReLU masks go
// to LDS, 16 bits per lane and accumulator tile), the head's adjoint seeds the last
// hidden layer, and every earlier adjoint is a chain of MFMAs with the transposed weight
// tiles (rows = a layer's inputs, contraction over its outputs) masked by the saved ReLU
// pattern.  The product with the transposed first layer leaves each lane holding the
// adjoints of exactly the Fourier features it encoded, so the chain rule through
// sin/cos ends in registers too.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "mlp_device.hpp"
#include "mlp_layout.hpp"
#include "grad_args.hpp"
#include "tuning.hpp"

namespace ddf {



namespace {

constexpr int kLdsBytes = 160 * 1024;



template <int P, int W, int NB, bool kTrain>
__global__ __launch_bounds__(NB == 2 ? 512 : 256) void grad_kernel(GradArgs a) {
    using Op = typename OpOf<P>::T;
    constexpr int NMB = W / 32;
    constexpr int KB = k_per_block(P);
    constexpr int NKB = W / KB;
    constexpr int K0 = layer0_kblocks(P);
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int64_t n = a.n;
    const bool multi = a.n_nets > 0;
    const int depth_max = a.depth;
    const int64_t count = a.count_dev ? min<int64_t>(*a.count_dev, n) : n;

    // single network: biases and head rows staged in LDS; multi: read from each blob (L2)
    float *s_bias = reinterpret_cast<float *>(smem);
    float *s_head = s_bias + (multi ? 0 : W * depth_max + 4);   // [2][W]
    uint16_t *s_mask = reinterpret_cast<uint16_t *>(s_head + (multi ? 0 : 2 * W));
    float *s_loss = reinterpret_cast<float *>(s_mask + (blockDim.x / 64) * depth_max * NMB * NB * 64);
    if (!multi) {
        const NetLayout L0 = make_layout(W, depth_max, P);
        for (int i = threadIdx.x; i < W * depth_max + 4; i += blockDim.x)
            s_bias[i] = reinterpret_cast<const float *>(a.blob + L0.bias_off)[i];
        for (int i = threadIdx.x; i < 2 * W; i += blockDim.x)
            s_head[i] = reinterpret_cast<const float *>(a.blob + L0.head_rows_off)[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int wpb = blockDim.x >> 6;
    uint16_t *wmask = s_mask + (int64_t)wave * depth_max * NMB * NB * 64;
    float loss_acc = 0.f;
    const float inv_n = (kTrain && a.loss_scalars) ? a.loss_scalars[0] : 0.f;
    const float inv_nhit = (kTrain && a.loss_scalars) ? a.loss_scalars[1] : 0.f;

    // work list: the tiles of every network segment, one after another
    const int nk = multi ? a.n_nets : 1;
    int64_t pre[kMaxNets + 1];
    pre[0] = 0;
#pragma unroll
    for (int k = 0; k < kMaxNets; ++k) {
        const int64_t cnt = k < nk ? (multi ? (int64_t)a.seg_count[k] : count) : 0;
        pre[k + 1] = pre[k] + (cnt + 32 * NB - 1) / (32 * NB);
    }
    const int64_t ntile = pre[kMaxNets];

    for (int64_t tile = (int64_t)blockIdx.x * wpb + wave; tile < ntile; tile += (int64_t)gridDim.x * wpb) {
        int k = 0;
        int64_t pk = 0;
#pragma unroll
        for (int i = 1; i < kMaxNets; ++i)
            if (tile >= pre[i] && i < nk) {
                k = i;
                pk = pre[i];
            }
        const uint8_t *blob = multi ? a.blobs[k] : a.blob;
        const int depth = multi ? a.depths[k] : a.depth;
        const NetLayout L = make_layout(W, depth, P);
        const uint8_t *gsrc = blob + L.grad_off;
        const float *bias_src = multi ? reinterpret_cast<const float *>(blob + L.bias_off) : s_bias;
        const float *head_src = multi ? reinterpret_cast<const float *>(blob + L.head_rows_off) : s_head;
        const int64_t seg_lo = multi ? (int64_t)a.seg_offset[k] : 0;
        const int64_t seg_end = seg_lo + (multi ? (int64_t)a.seg_count[k] : count);
        const int64_t base = seg_lo + (tile - pk) * 32 * NB;
        Op b[NKB][NB];
        float v[NB][kInRaw];
        bool valid[NB];
        // ---- encoding
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t r = base + nb * 32 + col;
            valid[nb] = r < seg_end;
#pragma unroll
            for (int j = 0; j < kInRaw; ++j) v[nb][j] = valid[nb] ? a.rays[(int64_t)j * n + r] : 0.f;
            float feat[kSlotsPerHalf];
            encode_var<P == kFP32>(h ? v[nb][3] : v[nb][0], feat);
            encode_var<P == kFP32>(h ? v[nb][4] : v[nb][1], feat + kFeatPerVar);
            encode_var<P == kFP32>(h ? 0.f : v[nb][2], feat + 2 * kFeatPerVar);
            feat[kSlotsPerHalf - 1] = 0.f;
            if constexpr (kTrain) {
                if (valid[nb]) {
#pragma unroll
                    for (int f = 0; f < kSlotsPerHalf - 1; ++f) {
                        const int c = feature_column(h, f);
                        if (c >= 0) a.ws_gamma[(int64_t)c * n + r] = feat[f];
                    }
                }
            }
            if constexpr (P == kBF16) {
                // layer-0 bias rides in two unused feature slots of lane half 1
                feat[kBiasSlot0] = h ? 1.f : feat[kBiasSlot0];
                feat[kBiasSlot1] = h ? 1.f : 0.f;
#pragma unroll
                for (int kb = 0; kb < K0; ++kb)
#pragma unroll
                    for (int s = 0; s < 8; ++s) b[kb][nb][s] = (__bf16)feat[kb * 8 + s];
            } else {
#pragma unroll
                for (int kb = 0; kb < K0; ++kb) b[kb][nb] = feat[kb];
            }
        }
        // ---- forward (ReLU masks to LDS)
        for (int l = 0; l < depth; ++l) {
            const int64_t t0 = L.layer_tile(l);
            f32x16 acc[NMB][NB];
            if (l == 0)
                mfma_tiles<P, NMB, NB, K0, NKB>(blob, t0, b, acc, lane);
            else
                mfma_tiles<P, NMB, NB, NKB, NKB>(blob, t0, b, acc, lane);
            if constexpr (P == kBF16) {
                if (l > 0) {   // bias K-block of a hidden layer
                    const Op one = bias_operand(h);
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb) {
                        const Op w = load_a<P>(blob, t0 + (int64_t)NKB * NMB + mb, lane);
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma<P>(w, one, acc[mb][nb]);
                    }
                }
            }
            const float *bias = bias_src + l * W;
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
                float bv[16];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const f32x4 b4 = P == kBF16 ? f32x4{0.f, 0.f, 0.f, 0.f}   // bf16: bias already accumulated
                                                : *reinterpret_cast<const f32x4 *>(bias + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                    for (int i = 0; i < 4; ++i) bv[4 * g + i] = b4[i];
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    if constexpr (P == kBF16 && !kTrain) {   // bias already accumulated; packed ReLU
                        uint32_t bits = 0;
#pragma unroll
                        for (int j = 0; j < 16; ++j) bits |= (acc[mb][nb][j] > 0.f ? 1u : 0u) << j;
                        wmask[((l * NMB + mb) * NB + nb) * 64 + lane] = (uint16_t)bits;
                        relu_tile_to_bf16(acc[mb][nb], mb, nb, b);
                        continue;
                    }
                    float y[16];
                    uint32_t bits = 0;
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        const float z = acc[mb][nb][j] + bv[j];
                        y[j] = fmaxf(z, 0.f);
                        bits |= (z > 0.f ? 1u : 0u) << j;
                    }
                    wmask[((l * NMB + mb) * NB + nb) * 64 + lane] = (uint16_t)bits;
                    if constexpr (kTrain) {
                        const int64_t r = base + nb * 32 + col;
                        if (valid[nb]) {
                            float *dst = a.ws_h + ((int64_t)l * W + mb * 32 + 4 * h) * n + r;
#pragma unroll
                            for (int j = 0; j < 16; ++j) dst[(int64_t)(8 * (j / 4) + (j % 4)) * n] = y[j];
                        }
                    }
                    tile_to_operands<P>(y, mb, nb, b);
                }
            }
        }
        // ---- head and seeds
        float gl[NB], gd[NB];
        {
            f32x16 acc[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < 16; ++j) acc[nb][j] = 0.f;
            const int64_t t0 = L.head_tile();
            {
                f32x16 hacc[1][NB];
                mfma_tiles<P, 1, NB, NKB, NKB>(blob, t0, b, hacc, lane);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb] = hacc[0][nb];
            }
            float hb0 = bias_src[W * depth], hb1 = bias_src[W * depth + 1];
            if constexpr (P == kBF16) {
                const Op w = load_a<P>(blob, t0 + NKB, lane);
                const Op one = bias_operand(h);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<P>(w, one, acc[nb]);
                hb0 = hb1 = 0.f;
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                // rows 0 (logit) and 1 (distance) live in lanes 0..31, plus rows 2 and 3 (the bf16
                // remainders of the head rows, zero in float32); share them with the upper half
                const float z = __shfl(acc[nb][0] + acc[nb][2], col) + hb0;
                const float dd = __shfl(acc[nb][1] + acc[nb][3], col) + hb1;
                const int64_t r = base + nb * 32 + col;
                if (h == 0 && valid[nb]) {
                    if (a.logit_out) a.logit_out[r] = z;
                    if (a.dist_out) a.dist_out[r] = dd;
                }
                if (kTrain && a.t_label) {
                    const float t = valid[nb] ? a.t_label[r] : INFINITY;
                    float g0, g1;
                    const float term = ray_loss(z, dd, t, inv_n, inv_nhit, a.loss, g0, g1);
                    gl[nb] = valid[nb] ? g0 : 0.f;
                    gd[nb] = valid[nb] ? g1 : 0.f;
                    if (h == 0 && valid[nb]) {
                        loss_acc += term;
                        a.ws_delta[(int64_t)depth * W * n + r] = gl[nb];
                        a.ws_delta[(int64_t)depth * W * n + n + r] = gd[nb];
                    }
                } else {
                    gl[nb] = (valid[nb] && a.g_logit_in) ? a.g_logit_in[(base + nb * 32 + col)] : 0.f;
                    gd[nb] = (valid[nb] && a.g_dist_in) ? a.g_dist_in[(base + nb * 32 + col)] : 0.f;
                    if (kTrain && h == 0 && valid[nb]) {
                        a.ws_delta[(int64_t)depth * W * n + r] = gl[nb];
                        a.ws_delta[(int64_t)depth * W * n + n + r] = gd[nb];
                    }
                }
            }
        }
        if (a.forward_only) continue;
        // ---- adjoint of the last hidden layer: head rows times the seeds, masked.  The
        // accumulator array carries each layer's adjoint (D layout) down the network.
        f32x16 acc[NMB][NB];
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) {
            float w0[16], w1[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const f32x4 a4 = *reinterpret_cast<const f32x4 *>(head_src + mb * 32 + 8 * g + 4 * h);
                const f32x4 b4 = *reinterpret_cast<const f32x4 *>(head_src + W + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    w0[4 * g + i] = a4[i];
                    w1[4 * g + i] = b4[i];
                }
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const uint32_t bits = wmask[(((depth - 1) * NMB + mb) * NB + nb) * 64 + lane];
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    acc[mb][nb][j] = ((bits >> j) & 1u) ? fmaf(gl[nb], w0[j], gd[nb] * w1[j]) : 0.f;
            }
        }
        // ---- adjoints of the hidden layers, top down
        for (int l = depth - 1; l >= 0; --l) {
            if constexpr (kTrain) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int64_t r = base + nb * 32 + col;
                    if (valid[nb]) {
#pragma unroll
                        for (int mb = 0; mb < NMB; ++mb) {
                            float *dst = a.ws_delta + ((int64_t)l * W + mb * 32 + 4 * h) * n + r;
#pragma unroll
                            for (int j = 0; j < 16; ++j) dst[(int64_t)(8 * (j / 4) + (j % 4)) * n] = acc[mb][nb][j];
                        }
                    }
                }
            }
            if (l == 0) break;
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    float y[16];
#pragma unroll
                    for (int j = 0; j < 16; ++j) y[j] = acc[mb][nb][j];
                    tile_to_operands<P>(y, mb, nb, b);
                }
            const int64_t t0 = L.grad_layer_tile(l);
            mfma_tiles<P, NMB, NB, NKB, NKB>(gsrc, t0, b, acc, lane);
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const uint32_t bits = wmask[(((l - 1) * NMB + mb) * NB + nb) * 64 + lane];
#pragma unroll
                    for (int j = 0; j < 16; ++j) acc[mb][nb][j] = ((bits >> j) & 1u) ? acc[mb][nb][j] : 0.f;
                }
        }
        if (!a.g_rays) continue;
        // ---- transposed first layer: adjoints of this lane's 48 feature slots
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                float y[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) y[j] = acc[mb][nb][j];
                tile_to_operands<P>(y, mb, nb, b);
            }
        f32x16 acc0[kGradRowBlocks0][NB];
        mfma_tiles<P, kGradRowBlocks0, NB, NKB, NKB>(gsrc, 0, b, acc0, lane);
        // ---- chain rule through the Fourier features
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t r = base + nb * 32 + col;
#pragma unroll
            for (int var = 0; var < 3; ++var) {
                if (h == 1 && var == 2) continue;
                float f[kFeatPerVar];
                const float x = h ? v[nb][3 + var] : v[nb][var];
                encode_var<P == kFP32>(x, f);
                float g = acc0[(var * kFeatPerVar) / 16][nb][(var * kFeatPerVar) % 16];
#pragma unroll
                for (int k = 0; k < kNFreq; ++k) {
                    const int fs = var * kFeatPerVar + 1 + k, fc = var * kFeatPerVar + 1 + kNFreq + k;
                    const float gs = acc0[fs / 16][nb][fs % 16], gc = acc0[fc / 16][nb][fc % 16];
                    g = fmaf((float)(1 << k), gs * f[1 + kNFreq + k] - gc * f[1 + k], g);
                }
                if (valid[nb]) a.g_rays[(int64_t)(h ? 3 + var : var) * n + r] = g;
            }
        }
    }
    if constexpr (kTrain) {
        // block sum of the loss terms -> one partial per block (summed in a fixed order later)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) loss_acc += __shfl_xor(loss_acc, off);
        if (lane == 0) s_loss[wave] = loss_acc;
        __syncthreads();
        if (threadIdx.x == 0 && a.loss_partial) {
            float t = 0.f;
            for (int w = 0; w < wpb; ++w) t += s_loss[w];
            a.loss_partial[blockIdx.x] = t;
        }
    }
}

int cu_count_grad() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    });
    return cus;
}

template <int P, int W, int NB, bool kTrain>
ddf_status launch_grad(const GradArgs &args, hipStream_t s, int grid_cap) {
    auto kern = grad_kernel<P, W, NB, kTrain>;
    static std::once_flag once;
    std::call_once(once, [&] { (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes); });
    const int threads = NB == 2 ? 512 : 256;
    const int wpb = threads / 64;
    const size_t lds = ((size_t)W * args.depth + 4 + 2 * W) * 4 + (size_t)wpb * args.depth * (W / 32) * NB * 64 * 2 + 16 * 4;
    const int64_t ntile = (args.n + 32 * NB - 1) / (32 * NB);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((ntile + wpb - 1) / wpb, grid_cap));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, s, args);
    return launch_status("ddf gradient kernel");
}

}  // namespace

// Shared with the training driver: grid size used for a given batch (loss partials).
int64_t grad_grid(int width, int precision, int64_t n) {
    if (precision == kFP32) return sweep_grid(width, n);   // training runs the LDS sweep
    const int NB = (width == 128 && precision != kFP32) ? 2 : 1;
    const int wpb = NB == 2 ? 8 : 4;
    const int64_t ntile = (n + 32 * NB - 1) / (32 * NB);
    return std::max<int64_t>(1, std::min<int64_t>((ntile + wpb - 1) / wpb,
                                                  (int64_t)cu_count_grad() * tuning(DDF_TUNE_GRAD_WG_PER_CU)));
}

ddf_status grad_dispatch(const ddf_net *net, const GradArgs &args, bool train, hipStream_t s) {
    const int cap = cu_count_grad() * tuning(DDF_TUNE_GRAD_WG_PER_CU);
    const int w = net->width, p = net->precision;
    if (train) {   // parameter gradients: float32 networks only (ddf_backward checks)
        DDF_REQUIRE(p == kFP32, DDF_ERR_UNSUPPORTED, "parameter gradients need a float32 network");
        if (!args.g_rays && args.n_nets == 0) return sweep_dispatch(w, args, s);
        return w == 128 ? launch_grad<kFP32, 128, 1, true>(args, s, cap) : launch_grad<kFP32, 256, 1, true>(args, s, cap);
    }
    if (p == kBF16) return stream_dispatch(w, args, s);   // weights streamed through LDS
    return w == 128 ? launch_grad<kFP32, 128, 1, false>(args, s, cap) : launch_grad<kFP32, 256, 1, false>(args, s, cap);
}

ddf_status grad_dispatch_multi(int width, int precision, const GradArgs &args, hipStream_t s) {
    DDF_REQUIRE(args.n_nets >= 1 && args.n_nets <= kMaxNets, DDF_ERR_UNSUPPORTED, "too many networks in one launch");
    const int cap = cu_count_grad() * tuning(DDF_TUNE_GRAD_WG_PER_CU);
    if (precision == kBF16) return stream_dispatch(width, args, s);
    return width == 128 ? launch_grad<kFP32, 128, 1, false>(args, s, cap) : launch_grad<kFP32, 256, 1, false>(args, s, cap);
}

}  // namespace ddf
