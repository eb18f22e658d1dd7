// Training sweep of a float32 network (Sec. V-A training, the hand-written backward): the
// forward pass with its side outputs, the loss seeds, and the adjoints of every hidden layer,
// for one network of width 128 or 256.
//
// A workgroup of eight waves takes 64 rays at a time and keeps their layer values in LDS
// ([ray][unit], float32): every wave reads the whole input of a layer from LDS as MFMA B
// operands (four K-steps per 16-byte read) and produces its own M-blocks (width 256: one
// 32-row block for both 32-ray halves; width 128: one block for one half), so no wave holds
// more than one layer's slice in registers.  Weight tiles come from the L2-resident blob
// (one 256-byte tile per wave and K-step, the layout the per-wave kernels read), ReLU masks
// go to LDS for the reverse sweep.  The layer products run over the same tiles and operands
// in the same order as the per-wave kernel; the head's two rows are summed in chunks of 16
// K-steps spread over all waves, so outputs and seeds agree with it to float32 rounding.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "grad_args.hpp"
#include "mlp_device.hpp"
#include "mlp_layout.hpp"

namespace ddf {
namespace {

constexpr int kSweepRays = 64;
constexpr int kSweepWaves = 8;
constexpr int kSweepLds = 160 * 1024;

template <int W>
struct SweepGeo {
    static constexpr int NMB = W / 32;
    static constexpr int NKB = W / 2;   // float32 K-steps of a hidden layer
    static constexpr int NBW = W == 256 ? 2 : 1;   // 32-ray blocks per wave
    static constexpr int XP = W + 4;                // row pitch of the LDS layer values (floats)
    static_assert(NMB * 2 == kSweepWaves * NBW, "every (M-block, ray block) pair has one wave");
};

template <int W>
__host__ __device__ inline size_t sweep_lds_bytes(int depth) {
    using G = SweepGeo<W>;
    return (size_t)kSweepRays * G::XP * 4                  // layer values
           + (size_t)depth * G::NMB * 2 * 64 * 2           // ReLU masks [layer][M-block][ray block][lane]
           + (size_t)2 * kSweepRays * 4                    // seeds
           + (size_t)4 * 2 * 2 * 32 * 4                    // head partial sums [chunk][ray block][row][col]
           + (size_t)kSweepWaves * 4;                      // loss partials
}

// One wave's products of a layer: KS K-steps of the tiles t0 + kb * nmb + mb against the
// layer values in LDS.  kFeat: layer 0 (K-step kb of lane half h reads feature slot
// 40 h + kb); otherwise K-step kb reads unit 32 (kb / 16) + 8 ((kb % 16) / 4) + 4 h + kb % 4,
// the contraction order of the packed tiles.
template <int W, int KS, bool kFeat>
__device__ __attribute__((always_inline)) inline void sweep_mfma(const uint8_t *blob, int64_t t0, int nmb, int mb,
                                                                 const float *X, int nb0, int lane,
                                                                 f32x16 (&acc)[SweepGeo<W>::NBW], int kb0 = 0) {
    using G = SweepGeo<W>;
    constexpr int NBW = G::NBW;
    static_assert(KS % 4 == 0, "K-steps come in groups of four");
    const int h = lane >> 5, col = lane & 31;
    const int64_t tstride = (int64_t)nmb * 64;   // floats between consecutive K-steps
    const float *tiles = reinterpret_cast<const float *>(blob) + (t0 + mb) * 64 + lane + kb0 * tstride;
    auto unit = [&](int kb) {
        kb += kb0;
        return kFeat ? 40 * h + kb : 32 * (kb / 16) + 8 * ((kb % 16) / 4) + 4 * h;
    };
    constexpr int kG = 4;   // groups of four K-steps of weight tiles in flight (L2 latency)
    float a[kG][4];
#pragma unroll
    for (int g = 0; g < kG - 1; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) a[g][q] = 4 * g < KS ? tiles[(4 * g + q) * tstride] : 0.f;
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) acc[nb] = f32x16{};
#pragma unroll 4
    for (int kb = 0; kb < KS; kb += 4) {
        if (kb + 4 * (kG - 1) < KS) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[kG - 1][q] = tiles[(kb + 4 * (kG - 1) + q) * tstride];
        }
        f32x4 b4[NBW];
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
            b4[nb] = *reinterpret_cast<const f32x4 *>(X + ((nb0 + nb) * 32 + col) * G::XP + unit(kb));
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb)
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][q], b4[nb][q], acc[nb], 0, 0, 0);
#pragma unroll
        for (int g = 0; g + 1 < kG; ++g)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[g][q] = a[g + 1][q];
    }
}

// Occupancy: at width 256 one workgroup per CU (two waves per SIMD, up to 256 registers: no
// spill); at width 128 two workgroups per CU (four waves per SIMD, 128 registers, which spills
// 176 bytes per lane of the head-chunk state).  Measured on MI355X, training step at batch
// 65,536: width 256 1.40 ms against 1.44 ms with two workgroups and the spill; width 128
// 0.46 ms with two workgroups and the spill against 0.51 ms with one and none.
template <int W>
constexpr int sweep_wg_per_cu() { return W == 256 ? 1 : 2; }

template <int W>
__global__ __launch_bounds__(kSweepWaves * 64, sweep_wg_per_cu<W>() * 2) void sweep_kernel(GradArgs a) {
    using G = SweepGeo<W>;
    constexpr int NMB = G::NMB, NKB = G::NKB, NBW = G::NBW, XP = G::XP;
    constexpr int K0 = layer0_kblocks(kFP32);
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int depth = a.depth;
    const int64_t n = a.n;
    const int64_t rstride = a.ray_stride ? a.ray_stride : n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int mb = W == 256 ? wave : wave >> 1;   // this wave's M-block
    const int nb0 = W == 256 ? 0 : (wave & 1);    // and its first ray block

    float *X = reinterpret_cast<float *>(smem);
    uint16_t *s_mask = reinterpret_cast<uint16_t *>(X + kSweepRays * XP);
    float *s_seed = reinterpret_cast<float *>(s_mask + depth * NMB * 2 * 64);   // [2][64]
    float *s_hpart = s_seed + 2 * kSweepRays;
    float *s_loss = s_hpart + 4 * 2 * 2 * 32;

    const NetLayout L = make_layout(W, depth, kFP32);
    const uint8_t *blob = a.blob;
    const float *bias = reinterpret_cast<const float *>(blob + L.bias_off);
    const float *head_rows = reinterpret_cast<const float *>(blob + L.head_rows_off);
    const float *gblob = reinterpret_cast<const float *>(blob + L.grad_off);
    const float inv_n = a.loss_scalars ? a.loss_scalars[0] : 0.f;
    const float inv_nhit = a.loss_scalars ? a.loss_scalars[1] : 0.f;
    float loss_acc = 0.f;
    const int64_t ntile = (n + kSweepRays - 1) / kSweepRays;

    auto mask_at = [&](int l, int nb) -> uint16_t & { return s_mask[((l * NMB + mb) * 2 + nb) * 64 + lane]; };
    // D-layout value j of this lane: unit mb * 32 + 8 (j / 4) + 4 h + j % 4 of ray block nb

    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t base = tile * kSweepRays;
        // ---- encoding: 64 rays x 5 variables, 13 feature slots each, into X[ray][40 h + slot]
        for (int t = threadIdx.x; t < kSweepRays * 6; t += blockDim.x) {
            const int ray = t % kSweepRays, grp = t / kSweepRays;   // grp: 3 h + variable slot group
            const int hh = grp / 3, g = grp % 3;
            const int64_t r = base + ray;
            const bool valid = r < n;
            float *dst = X + ray * XP + 40 * hh + kFeatPerVar * g;
            if (hh == 1 && g == 2) {   // the unused slot group of lane half 1, and the pad slot
#pragma unroll
                for (int f = 0; f < kFeatPerVar + 1; ++f) dst[f] = 0.f;
                continue;
            }
            const int var = hh ? 3 + g : g;
            const float x = valid ? a.rays[(int64_t)var * rstride + r] : 0.f;
            float feat[kFeatPerVar];
            encode_var<true>(x, feat);
#pragma unroll
            for (int f = 0; f < kFeatPerVar; ++f) {
                dst[f] = valid ? feat[f] : 0.f;
                const int c = feature_column(hh, kFeatPerVar * g + f);
                if (valid && c >= 0 && a.ws_gamma) a.ws_gamma[(int64_t)c * n + r] = feat[f];
            }
            if (hh == 0 && g == 2) dst[kFeatPerVar] = 0.f;   // pad slot 39 of lane half 0
        }
        __syncthreads();
        // ---- forward: X holds the layer input; every wave reads it, then writes its slice
        for (int l = 0; l < depth; ++l) {
            f32x16 acc[NBW];
            if (l == 0)
                sweep_mfma<W, K0, true>(blob, L.layer_tile(0), NMB, mb, X, nb0, lane, acc);
            else
                sweep_mfma<W, NKB, false>(blob, L.layer_tile(l), NMB, mb, X, nb0, lane, acc);
            __syncthreads();   // the input is read by every wave before anyone overwrites it
            float bv[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const f32x4 b4 = *reinterpret_cast<const f32x4 *>(bias + l * W + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                for (int i = 0; i < 4; ++i) bv[4 * g + i] = b4[i];
            }
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int ray = (nb0 + nb) * 32 + col;
                const int64_t r = base + ray;
                float y[16];
                uint32_t bits = 0;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const float z = acc[nb][j] + bv[j];
                    y[j] = fmaxf(z, 0.f);
                    bits |= (z > 0.f ? 1u : 0u) << j;
                }
                mask_at(l, nb0 + nb) = (uint16_t)bits;
                if (r < n && a.ws_h) {
                    float *dst = a.ws_h + ((int64_t)l * W + mb * 32 + 4 * h) * n + r;
#pragma unroll
                    for (int j = 0; j < 16; ++j) dst[(int64_t)(8 * (j / 4) + (j % 4)) * n] = y[j];
                }
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    *reinterpret_cast<f32x4 *>(X + ray * XP + mb * 32 + 8 * g + 4 * h) =
                        f32x4{y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
            }
            __syncthreads();
        }
        // ---- head (rows 0 and 1 of its one M-block) in four chunks of its K-steps (width 256:
        // waves 0-3, each for both ray blocks; width 128: chunk = M-block index, every ray
        // block); the partial sums meet in LDS (their 2 KiB keep two workgroups per CU at depth
        // 6) and the waves of M-block 0 add them in chunk order and form the loss seeds
        constexpr int kChunks = 4, kChunkK = NKB / kChunks;
        if (W == 128 || wave < kChunks) {
            const int chunk = W == 256 ? wave : mb;
            f32x16 hacc[NBW];
            sweep_mfma<W, kChunkK, false>(blob, L.head_tile(), 1, 0, X, nb0, lane, hacc, chunk * kChunkK);
            if (h == 0) {
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) {
                    float *hp = s_hpart + ((chunk * 2 + nb0 + nb) * 2) * 32 + col;
                    hp[0] = hacc[nb][0];    // row 0: logit
                    hp[32] = hacc[nb][1];   // row 1: distance
                }
            }
        }
        __syncthreads();
        if (mb == 0) {
            const float hb0 = bias[W * depth], hb1 = bias[W * depth + 1];
            // head output `row` (0: logit, 1: distance) of ray col of ray block blk
            auto head_sum = [&](int blk, int row) {
                float v = 0.f;
#pragma unroll
                for (int c = 0; c < kChunks; ++c) v += s_hpart[((c * 2 + blk) * 2 + row) * 32 + col];
                return v + (row ? hb1 : hb0);
            };
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int blk = nb0 + nb;
                const int ray = blk * 32 + col;
                const int64_t r = base + ray;
                const bool valid = r < n;
                const float z = head_sum(blk, 0), dd = head_sum(blk, 1);
                float gl = 0.f, gd = 0.f;
                if (a.eik_n > 0) {
                    // directed Eikonal pairs: block 0 holds rays base / 2 + col, block 1 the same
                    // rays moved by h along their directions; residual r = (d(x + h d) - d(x)) / h + 1
                    const int64_t i = base / 2 + col;
                    const bool ok = i < a.eik_n;
                    const float t = ok ? a.t_label[i] : INFINITY;
                    const float d_at = blk == 0 ? dd : head_sum(0, 1), d_moved = blk == 0 ? head_sum(1, 1) : dd;
                    const bool on = ok && t < INFINITY && t > a.eik_h;
                    const float res = on ? (d_moved - d_at) / a.eik_h + 1.f : 0.f;
                    const float g = 2.f * a.eik_lam * res * inv_n / a.eik_h;
                    if (blk == 0) {
                        float g0, g1;
                        const float term = ray_loss(z, dd, t, inv_n, inv_nhit, a.loss, g0, g1);
                        gl = ok ? g0 : 0.f;
                        gd = ok ? g1 - g : 0.f;
                        if (h == 0 && ok) loss_acc += term + a.eik_lam * res * res * inv_n;
                    } else {
                        gd = g;
                    }
                } else if (a.t_label) {
                    const float t = valid ? a.t_label[r] : INFINITY;
                    float g0, g1;
                    const float term = ray_loss(z, dd, t, inv_n, inv_nhit, a.loss, g0, g1);
                    gl = valid ? g0 : 0.f;
                    gd = valid ? g1 : 0.f;
                    if (h == 0 && valid) loss_acc += term;
                } else {
                    gl = (valid && a.g_logit_in) ? a.g_logit_in[r] : 0.f;
                    gd = (valid && a.g_dist_in) ? a.g_dist_in[r] : 0.f;
                }
                if (h == 0) {
                    if (valid) {
                        // a query with a NaN input gives NaN outputs (the ReLUs would hide it)
                        bool nan_ray = false;
#pragma unroll
                        for (int j = 0; j < kInRaw; ++j) nan_ray |= isnan(a.rays[(int64_t)j * rstride + r]);
                        if (a.logit_out) a.logit_out[r] = nan_ray ? NAN : z;
                        if (a.dist_out) a.dist_out[r] = nan_ray ? NAN : dd;
                        if (a.ws_delta) {
                            a.ws_delta[(int64_t)depth * W * n + r] = gl;
                            a.ws_delta[(int64_t)depth * W * n + n + r] = gd;
                        }
                    }
                    s_seed[ray] = gl;
                    s_seed[kSweepRays + ray] = gd;
                }
            }
        }
        __syncthreads();
        if (a.forward_only) continue;
        // ---- adjoint of the last hidden layer: head rows times the seeds, masked
        {
            float w0[16], w1[16];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const f32x4 a4 = *reinterpret_cast<const f32x4 *>(head_rows + mb * 32 + 8 * g + 4 * h);
                const f32x4 b4 = *reinterpret_cast<const f32x4 *>(head_rows + W + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    w0[4 * g + i] = a4[i];
                    w1[4 * g + i] = b4[i];
                }
            }
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int ray = (nb0 + nb) * 32 + col;
                const int64_t r = base + ray;
                const float gl = s_seed[ray], gd = s_seed[kSweepRays + ray];
                const uint32_t bits = mask_at(depth - 1, nb0 + nb);
                float y[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) y[j] = ((bits >> j) & 1u) ? fmaf(gl, w0[j], gd * w1[j]) : 0.f;
                if (r < n) {
                    float *dst = a.ws_delta + ((int64_t)(depth - 1) * W + mb * 32 + 4 * h) * n + r;
#pragma unroll
                    for (int j = 0; j < 16; ++j) dst[(int64_t)(8 * (j / 4) + (j % 4)) * n] = y[j];
                }
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    *reinterpret_cast<f32x4 *>(X + ray * XP + mb * 32 + 8 * g + 4 * h) =
                        f32x4{y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
            }
        }
        __syncthreads();
        // ---- transposed hidden layers from the top: X holds layer l's adjoint
        for (int l = depth - 1; l >= 1; --l) {
            f32x16 acc[NBW];
            sweep_mfma<W, NKB, false>(reinterpret_cast<const uint8_t *>(gblob), L.grad_layer_tile(l), NMB, mb, X, nb0,
                                      lane, acc);
            __syncthreads();
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
                const int ray = (nb0 + nb) * 32 + col;
                const int64_t r = base + ray;
                const uint32_t bits = mask_at(l - 1, nb0 + nb);
                float y[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) y[j] = ((bits >> j) & 1u) ? acc[nb][j] : 0.f;
                if (r < n) {
                    float *dst = a.ws_delta + ((int64_t)(l - 1) * W + mb * 32 + 4 * h) * n + r;
#pragma unroll
                    for (int j = 0; j < 16; ++j) dst[(int64_t)(8 * (j / 4) + (j % 4)) * n] = y[j];
                }
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    *reinterpret_cast<f32x4 *>(X + ray * XP + mb * 32 + 8 * g + 4 * h) =
                        f32x4{y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
            }
            __syncthreads();
        }
    }
    // block sum of the loss terms -> one partial per block (summed in a fixed order later)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) loss_acc += __shfl_xor(loss_acc, off);
    if (lane == 0) s_loss[wave] = loss_acc;
    __syncthreads();
    if (threadIdx.x == 0 && a.loss_partial) {
        float t = 0.f;
        for (int w = 0; w < kSweepWaves; ++w) t += s_loss[w];
        a.loss_partial[blockIdx.x] = t;
    }
}

int cu_count_sweep() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    });
    return cus;
}

template <int W>
ddf_status launch_sweep(const GradArgs &a, hipStream_t s) {
    auto kern = sweep_kernel<W>;
    static std::once_flag once;
    std::call_once(once, [&] { (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kSweepLds); });
    const size_t lds = sweep_lds_bytes<W>(a.depth);
    DDF_REQUIRE(lds <= (size_t)kSweepLds, DDF_ERR_UNSUPPORTED, "training sweep: network too deep");
    hipLaunchKernelGGL(kern, dim3((unsigned)sweep_grid(W, a.n)), dim3(kSweepWaves * 64), lds, s, a);
    return launch_status("ddf training sweep");
}

}  // namespace

// Workgroups of the training sweep for n rays (each writes one loss partial): one per CU at
// width 256, two at width 128.
int64_t sweep_grid(int width, int64_t n) {
    const int64_t tiles = (n + kSweepRays - 1) / kSweepRays;
    const int per_cu = width == 256 ? sweep_wg_per_cu<256>() : sweep_wg_per_cu<128>();
    return std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)cu_count_sweep() * per_cu));
}

// Float32 training sweep of one network (no input gradient): features, activations, adjoints,
// head seeds and loss partials, as the per-wave gradient kernel writes them.
ddf_status sweep_dispatch(int width, const GradArgs &a, hipStream_t s) {
    DDF_REQUIRE(a.n_nets == 0 && !a.g_rays && a.depth >= 1 && a.depth <= 8, DDF_ERR_UNSUPPORTED,
                "training sweep: one network, no input gradient");
    return width == 256 ? launch_sweep<256>(a, s) : launch_sweep<128>(a, s);
}

}  // namespace ddf
