// The paper's own network (Sec. V-A): `depth` weight-normalised hidden ReLU layers of 512
// units on the raw oriented point (ox, oy, oz, polar angle, azimuth), one affine output (the
// field value), dropout the identity at query time; trained on the clamp loss (Eq. 7) or the
// squish loss (Eq. 6).
//
// Packing folds the weight normalisation, W = g v / |v| per row, on the device, into one of
// two blobs:
//   bf16 (queries, normals): the first layer as float32 tiles of the 32x32x2 float32 MFMA (the
//     five raw inputs and the bias are its six contraction slots: a raw coordinate rounded to
//     bf16 would move by up to 2^-9 of its size); the hidden layers as bf16 tiles of the
//     32x32x16 MFMA, their biases in float32 (each M-block's accumulation starts from its
//     bias); the output row as rows 0 and 1 of one 32-row block (the bf16 row and its bf16
//     remainder); the transposed tiles of the input gradient; the output row in float32.
//   float32 (training, float32 queries): float32 tiles of the 32x32x2 MFMA for every layer and
//     its transpose, biases in float32.
//
// bf16 kernel (paper_stream_kernel): a 512-wide layer of 32 rays is 32 KiB of bf16 operands, so
// a wave keeps one layer's input and one layer's output in registers (256 of its 512) and runs
// alone on its SIMD: a workgroup is four waves = 128 rays.  Weights stream through an LDS ring
// that all four waves read: one phase is one half of a 32-row M-block (16 K-blocks), two
// phases per barrier, four 16 KiB stages, each phase's tiles fetched two phases ahead by loads
// that write LDS directly; the first layer's tiles and the hidden biases stay in LDS.  Layer outputs stay in the accumulators and become the next layer's B operands
// (the contraction index renumbered in the packed tiles); ReLU masks go to LDS for the
// reverse sweep of the input gradient.
#include <cmath>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "grad_args.hpp"
#include "loss_device.hpp"
#include "mlp_device.hpp"
#include "mlp_layout.hpp"

namespace ddf {
namespace {

constexpr int kPW = 512;            // width
constexpr int kPNMB = kPW / 32;     // 32-row M-blocks
constexpr int kPNKB = kPW / 16;     // bf16 K-blocks of a hidden layer
constexpr int kPF32K = kPW / 2;     // float32 K-steps of a hidden layer
constexpr int kPK0 = 3;             // float32 K-steps of the first layer: (x, y), (z, theta), (phi, 1)
constexpr int kPMaxDepth = 8;

// Blob of one precision (byte offsets).
struct PaperLayout {
    int depth, prec;
    int64_t l0_off;       // float32 first-layer tiles [M-block][K-step][lane] (both precisions)
    int64_t hid_off;      // bf16: [(l - 1) * 16 + mb][32 K-blocks][lane][8]; fp32: [(l - 1)][256 kb][16 mb][lane]
    int64_t head_off;     // bf16: [32 K-blocks][lane][8]; fp32: [256 kb][lane] (row 0 = the output row)
    int64_t tr_off;       // transposed hidden layers as hid_off without bias blocks, then the
                          // transposed first layer (bf16: [32 kb]; fp32: [256 kb]; rows 0..4 = inputs)
    int64_t bias_off;     // hidden biases [(depth - 1)][512], float32
    int64_t row_off;      // the output row [512] and its bias [1], float32
    int64_t bytes;
};

__host__ __device__ inline PaperLayout paper_layout(int depth, int prec) {
    PaperLayout L;
    L.depth = depth;
    L.prec = prec;
    const int64_t nh = depth - 1;
    L.l0_off = 0;
    L.hid_off = (int64_t)kPNMB * kPK0 * 256;
    if (prec == kBF16) {
        L.head_off = L.hid_off + nh * kPNMB * kPNKB * 1024;
        L.tr_off = L.head_off + (int64_t)kPNKB * 1024;
        L.bias_off = L.tr_off + (nh * kPNMB * kPNKB + kPNKB) * 1024;
    } else {
        L.head_off = L.hid_off + nh * kPF32K * kPNMB * 256;
        L.tr_off = L.head_off + (int64_t)kPF32K * 256;
        L.bias_off = L.tr_off + (nh * kPF32K * kPNMB + kPF32K) * 256;
    }
    L.row_off = L.bias_off + nh * kPW * 4;
    L.bytes = L.row_off + (kPW + 4) * 4;
    return L;
}

// ------------------------------------------------------------------------------ packing
// Flat parameters: per hidden layer l, v_l [512][in_l], g_l [512], b_l [512] (in_0 = 5), then
// the output row [512] and its bias.
__host__ __device__ inline int64_t paper_layer_off(int l) {
    return l == 0 ? 0 : (int64_t)kPW * kInRaw + 2 * kPW + (int64_t)(l - 1) * ((int64_t)kPW * kPW + 2 * kPW);
}
__host__ __device__ inline int64_t paper_params(int depth) { return paper_layer_off(depth) + kPW + 1; }
__host__ __device__ inline int paper_in(int l) { return l == 0 ? kInRaw : kPW; }
// Plain (folded-weight) gradients: per layer [512][in_l] then [512]; the output layer [512], [1].
__host__ __device__ inline int64_t gw_layer_off(int l) {
    return l == 0 ? 0 : (int64_t)kPW * kInRaw + kPW + (int64_t)(l - 1) * ((int64_t)kPW * kPW + kPW);
}
__host__ __device__ inline int64_t gw_floats(int depth) { return gw_layer_off(depth) + kPW + 1; }

// Float-float numbers (hi + lo, |lo| <= half an ulp of hi) on the error-free transforms of
// Knuth (the rounding error of a sum) and Dekker (of a product, here by one fused
// multiply-add): about 48 significant bits from float32 arithmetic alone, so that the fold
// below rounds to the float32 nearest the exact weight without float64 on the GPU.  The
// transforms need every sum and product rounded as written: contraction of a product into a
// neighbouring sum (the compiler's default) is switched off inside them.
struct FF {
    float hi, lo;
};
__device__ inline FF ff_two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline FF ff_fast_two_sum(float a, float b) {   // |a| >= |b|
#pragma clang fp contract(off)
    const float s = a + b;
    return {s, b - (s - a)};
}
__device__ inline FF ff_two_prod(float a, float b) {
#pragma clang fp contract(off)
    const float p = a * b;
    return {p, fmaf(a, b, -p)};
}
__device__ inline FF ff_add(FF x, FF y) {
#pragma clang fp contract(off)
    const FF s = ff_two_sum(x.hi, y.hi);
    return ff_fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}
// sqrt(x) for x = hi + lo > 0: one Newton correction of the float32 root.
__device__ inline FF ff_sqrt(FF x) {
#pragma clang fp contract(off)
    const float r = sqrtf(x.hi);
    const FF rr = ff_two_prod(r, r);
    return ff_fast_two_sum(r, (((x.hi - rr.hi) - rr.lo) + x.lo) / (2.f * r));
}
// (a b) / d rounded to float32, for float32 a, b and float-float d > 0: a quotient and one
// correction from the exact remainder.
__device__ inline float ff_mul_div(float a, float b, FF d) {
#pragma clang fp contract(off)
    const FF n = ff_two_prod(a, b);
    const float q = n.hi / d.hi;
    const FF qd = ff_two_prod(q, d.hi);
    const float rem = (((n.hi - qd.hi) - qd.lo) + n.lo) - q * d.lo;
    return q + rem / d.hi;
}

// Row norms of the weight normalisation, norm[l][i] = |v_l[i, :]| as a float-float pair (one
// wave per row: float-float partial sums of the exact squares, added in a fixed lane order).
// The folded weight W = g v / |v| is formed to about 48 bits and rounded once to float32, so
// the bf16 rounding of a weight is decided from the float32 nearest the exact value, whatever
// order the norm was summed in (a float32 fold flips the float32 value of ~3e-5 of the weights,
// and each flip can move the bf16 rounding of that weight for every ray).
__global__ void paper_norm_kernel(const float *__restrict__ params, int depth, FF *__restrict__ norm) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row >= (int64_t)depth * kPW) return;
    const int l = (int)(row / kPW), i = (int)(row % kPW);
    const int in = paper_in(l);
    const float *v = params + paper_layer_off(l) + (int64_t)i * in;
    FF s{0.f, 0.f};
    for (int k = lane; k < in; k += 64) s = ff_add(s, ff_two_prod(v[k], v[k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = ff_add(s, FF{__shfl_xor(s.hi, off), __shfl_xor(s.lo, off)});
    if (lane == 0) norm[row] = ff_sqrt(s);
}

// Folded weight W_l[i][k] = (g_l[i] v_l[i][k]) / |v_l[i, :]|, rounded to float32.
__device__ inline float paper_w(const float *params, const FF *norm, int l, int i, int k) {
    const int in = paper_in(l);
    const float g = params[paper_layer_off(l) + (int64_t)kPW * in + i];
    return ff_mul_div(g, params[paper_layer_off(l) + (int64_t)i * in + k], norm[(int64_t)l * kPW + i]);
}
__device__ inline float paper_b(const float *params, int l, int i) {
    return params[paper_layer_off(l) + (int64_t)kPW * paper_in(l) + kPW + i];
}

// Float32 first-layer slot: M-block mb, K-step ks, lane -> W0[row][2 ks + lane / 32] (slot 5 = bias).
__device__ inline float l0_slot(const float *params, const FF *scale, int mb, int ks, int lane) {
    const int row = mb * 32 + (lane & 31), k = 2 * ks + (lane >> 5);
    return k < kInRaw ? paper_w(params, scale, 0, row, k) : paper_b(params, 0, row);
}

// One thread per packed element.
__global__ void paper_pack_kernel(const float *__restrict__ params, const FF *__restrict__ scale, int depth, int prec,
                                  uint8_t *__restrict__ blob) {
    const PaperLayout L = paper_layout(depth, prec);
    const int nh = depth - 1;
    const int64_t n_l0 = (int64_t)kPNMB * kPK0 * 64;
    int64_t n_hid, n_head, n_tr, n_bias;
    if (prec == kBF16) {
        n_hid = (int64_t)nh * kPNMB * kPNKB * 512;
        n_head = (int64_t)kPNKB * 512;
        n_tr = ((int64_t)nh * kPNMB * kPNKB + kPNKB) * 512;
        n_bias = (int64_t)nh * kPW;
    } else {
        n_hid = (int64_t)nh * kPF32K * kPNMB * 64;
        n_head = (int64_t)kPF32K * 64;
        n_tr = ((int64_t)nh * kPF32K * kPNMB + kPF32K) * 64;
        n_bias = (int64_t)nh * kPW;
    }
    const int64_t n_row = kPW + 4;
    const int64_t total = n_l0 + n_hid + n_head + n_tr + n_bias + n_row;
    const float *head_row = params + paper_layer_off(depth);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e;
        if (r < n_l0) {
            const int lane = (int)(r % 64), ks = (int)((r / 64) % kPK0), mb = (int)(r / (64 * kPK0));
            reinterpret_cast<float *>(blob + L.l0_off)[r] = l0_slot(params, scale, mb, ks, lane);
            continue;
        }
        r -= n_l0;
        if (prec == kBF16) {
            uint16_t *dst = nullptr;
            float w = 0.f;
            if (r < n_hid) {
                // tile ((l - 1) * 16 + mb) * 32 + kb, lane, slot s: row mb * 32 + lane % 32 of layer l
                const int s = (int)(r % 8), lane = (int)((r / 8) % 64);
                const int64_t t = r / 512;
                const int kb = (int)(t % kPNKB), mb = (int)((t / kPNKB) % kPNMB);
                const int l = 1 + (int)(t / ((int64_t)kPNKB * kPNMB));
                w = paper_w(params, scale, l, mb * 32 + (lane & 31), prev_unit(kBF16, kb, lane >> 5, s));
                dst = reinterpret_cast<uint16_t *>(blob + L.hid_off) + r;
            } else if ((r -= n_hid) < n_head) {
                // rows 0 and 1: the output row as bf16 and its bf16 remainder
                const int s = (int)(r % 8), lane = (int)((r / 8) % 64), kb = (int)(r / 512);
                const int row = lane & 31, h = lane >> 5;
                if (row < 2) {
                    const float x = head_row[prev_unit(kBF16, kb, h, s)];
                    const float hi = (float)(__bf16)x;
                    w = row == 0 ? hi : x - hi;
                }
                dst = reinterpret_cast<uint16_t *>(blob + L.head_off) + r;
            } else if ((r -= n_head) < n_tr) {
                // transposed layer l: A[m][k] = W_l[k][m], rows m = inputs of layer l; the
                // transposed first layer (the last 32 tiles) has rows 0..4 = the raw inputs
                const int s = (int)(r % 8), lane = (int)((r / 8) % 64);
                const int64_t t = r / 512;
                const int h = lane >> 5;
                if (t < (int64_t)nh * kPNMB * kPNKB) {
                    const int kb = (int)(t % kPNKB), mb = (int)((t / kPNKB) % kPNMB);
                    const int l = 1 + (int)(t / ((int64_t)kPNKB * kPNMB));
                    w = paper_w(params, scale, l, prev_unit(kBF16, kb, h, s), mb * 32 + (lane & 31));
                } else {
                    const int kb = (int)(t - (int64_t)nh * kPNMB * kPNKB), m = lane & 31;
                    if (m < kInRaw) w = paper_w(params, scale, 0, prev_unit(kBF16, kb, h, s), m);
                }
                dst = reinterpret_cast<uint16_t *>(blob + L.tr_off) + r;
            } else if ((r -= n_tr) < n_bias) {
                reinterpret_cast<float *>(blob + L.bias_off)[r] = paper_b(params, 1 + (int)(r / kPW), (int)(r % kPW));
                continue;
            } else {
                r -= n_bias;
                reinterpret_cast<float *>(blob + L.row_off)[r] =
                    r < kPW ? head_row[r] : (r == kPW ? head_row[kPW] : 0.f);
                continue;
            }
            *dst = bf16_bits(w);
            continue;
        }
        // float32 tiles: lane slot of K-step kb reads unit prev_unit(kFP32, kb, h, 0)
        if (r < n_hid) {
            const int lane = (int)(r % 64);
            const int64_t t = r / 64;
            const int mb = (int)(t % kPNMB), kb = (int)((t / kPNMB) % kPF32K);
            const int l = 1 + (int)(t / ((int64_t)kPNMB * kPF32K));
            reinterpret_cast<float *>(blob + L.hid_off)[r] =
                paper_w(params, scale, l, mb * 32 + (lane & 31), prev_unit(kFP32, kb, lane >> 5, 0));
            continue;
        }
        r -= n_hid;
        if (r < n_head) {
            const int lane = (int)(r % 64), kb = (int)(r / 64);
            reinterpret_cast<float *>(blob + L.head_off)[r] =
                (lane & 31) == 0 ? head_row[prev_unit(kFP32, kb, lane >> 5, 0)] : 0.f;
            continue;
        }
        r -= n_head;
        if (r < n_tr) {
            const int lane = (int)(r % 64), h = lane >> 5, m = lane & 31;
            const int64_t t = r / 64;
            float w = 0.f;
            if (t < (int64_t)nh * kPF32K * kPNMB) {
                const int mb = (int)(t % kPNMB), kb = (int)((t / kPNMB) % kPF32K);
                const int l = 1 + (int)(t / ((int64_t)kPNMB * kPF32K));
                w = paper_w(params, scale, l, prev_unit(kFP32, kb, h, 0), mb * 32 + m);
            } else {
                const int kb = (int)(t - (int64_t)nh * kPF32K * kPNMB);
                if (m < kInRaw) w = paper_w(params, scale, 0, prev_unit(kFP32, kb, h, 0), m);
            }
            reinterpret_cast<float *>(blob + L.tr_off)[r] = w;
            continue;
        }
        r -= n_tr;
        if (r < n_bias) {
            reinterpret_cast<float *>(blob + L.bias_off)[r] = paper_b(params, 1 + (int)(r / kPW), (int)(r % kPW));
            continue;
        }
        r -= n_bias;
        reinterpret_cast<float *>(blob + L.row_off)[r] = r < kPW ? head_row[r] : (r == kPW ? head_row[kPW] : 0.f);
    }
}

// ------------------------------------------------------------------------------ bf16 kernel
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(1))) const uint8_t gbl_u8;

constexpr int kPWaves = 4;
constexpr int kPRays = 32 * kPWaves;       // rays per workgroup tile
constexpr int kPStages = 4;
constexpr int kPStageBytes = 16 * 1024;    // half an M-block: 16 K-blocks
constexpr int kPAR = 4;                    // A tiles read ahead from LDS
constexpr int kPLds = 160 * 1024;

struct PLds {   // byte offsets of the LDS sections
    int l0, ring, bias, row, mask, bytes;
};
__host__ __device__ inline PLds paper_lds(int depth, bool grad) {
    PLds s;
    s.l0 = 0;
    s.ring = kPNMB * kPK0 * 256;
    s.bias = s.ring + kPStages * kPStageBytes;
    s.row = s.bias + (depth - 1) * kPW * 4;
    s.mask = s.row + (kPW + 4) * 4;
    s.bytes = s.mask + (grad ? kPWaves * depth * kPNMB * 64 * 2 : 0);
    return s;
}

// Phase q of a tile's program -> byte offset of its 16 tiles in the blob: the hidden layers
// (l, mb, half) and the output row's two halves lie back to back (phase q at hid_off + q x 16
// KiB), then for gradients the transposed hidden layers from the top and the transposed first
// layer.  Selects instead of branches: the fetch runs between MFMAs of a wave that is alone on
// its SIMD, where every taken branch idles the matrix core.
__device__ inline int paper_phase_off(const PaperLayout &L, int q) {
    const int nh = L.depth - 1;
    const int nfw = 32 * nh + 2;   // phases of the forward program
    const int q2 = q - nfw;
    // transposed hidden layer from the top: (nh - 1 - q2 / 32) x 512 + (q2 % 32) x 16 KiB; past
    // them the transposed first layer: nh x 512 + (q2 - 32 nh) x 16 KiB
    const int last = -(int)(q2 >= 32 * nh);   // all ones in the transposed first layer
    const int tr_kib = (((nh - 1 - (q2 >> 5)) * 512 + (q2 & 31) * 16) & ~last) | ((nh * 512 + (q2 - 32 * nh) * 16) & last);
    const int fw = -(int)(q < nfw);
    return (((int)L.hid_off + q * 16384) & fw) | (((int)L.tr_off + tr_kib * 1024) & ~fw);
}

// The ring of one workgroup: global phase counter g (phase g % NP of the workgroup's tile
// g / NP), phases beyond `gend` do not exist.  The blob is read through a buffer resource
// (loads past its end return zero instead of faulting).
struct PRing {
    __amdgpu_buffer_rsrc_t blob;
    PaperLayout L;
    int np;          // phases per tile
    int qf;          // phase within its tile of the next phase to fetch, (g + 2) % np
    int64_t gend;    // phases of this workgroup
    int64_t g;       // current phase
};

// This wave's share of phase gq's 16 tiles (q = gq % np, kept by the caller), loaded straight
// into its stage (16 bytes per lane: one instruction moves a whole 1 KiB tile): tiles wave,
// wave + 4, wave + 8, wave + 12.  Buffer loads that write LDS (not the global form) keep the
// compiler's waits for the ring's LDS reads exact: after a global load into LDS it waits for
// every outstanding LDS read instead of only the one an MFMA needs.
__device__ inline void paper_fetch(const PRing &rg, int64_t gq, int q, lds_u8 *ring, int wave, int lane) {
    if (gq >= rg.gend) return;   // wave-uniform
    const int off = paper_phase_off(rg.L, q);
    lds_u8 *stage = ring + (int)((uint32_t)gq % kPStages) * kPStageBytes;
#pragma unroll
    for (int j = 0; j < 16 / kPWaves; ++j) {
        const int i = wave + kPWaves * j;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rg.blob, (__attribute__((address_space(3))) void *)(stage + i * 1024),
                                                 16, off + i * 1024 + lane * 16, 0, 0, 0);
    }
}

// Fetches phase g + 2 and advances the fetch phase index.
__device__ inline void paper_fetch_next(PRing &rg, lds_u8 *ring, int wave, int lane) {
    paper_fetch(rg, rg.g + 2, rg.qf, ring, wave, lane);
    rg.qf = rg.qf + 1 == rg.np ? 0 : rg.qf + 1;
}

// The LDS writes of the buffer loads are not tracked by the compiler: wait for them (vmcnt(0))
// before the barrier that publishes a stage.
__device__ inline void paper_stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ inline bf16x8 ptile(const lds_u8 *stage, int i, int lane) {
    return *reinterpret_cast<const __attribute__((address_space(3))) bf16x8 *>(stage + i * 1024 + lane * 16);
}

struct PAR {
    bf16x8 r[kPAR];
};

// One phase's MFMA chain over K-blocks kb0 .. kb0 + KS - 1 of `bin`, accumulating into acc.
// kLoadFirst: the ring does not hold this phase's first tiles yet; kNext: the last steps read
// the next phase's first tiles (its stage is already published).
template <int KS, int kb0, bool kLoadFirst, bool kNext>
__device__ __attribute__((always_inline)) inline void pchain(const lds_u8 *st, const lds_u8 *st_next, PAR &ar,
                                                             const bf16x8 (&bin)[kPNKB][1], f32x16 &acc, int lane) {
    if constexpr (kLoadFirst) {
#pragma unroll
        for (int j = 0; j < kPAR; ++j) ar.r[j] = ptile(st, j, lane);
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 a = ar.r[ks % kPAR];
        if (ks + kPAR < KS) ar.r[ks % kPAR] = ptile(st, ks + kPAR, lane);
        else if (kNext) ar.r[ks % kPAR] = ptile(st_next, ks + kPAR - KS, lane);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bin[kb0 + ks][0], acc, 0, 0, 0);
    }
    if constexpr (kNext) {   // the next phase's tile j landed in slot (KS + j) % kPAR
        PAR t = ar;
#pragma unroll
        for (int j = 0; j < kPAR; ++j) ar.r[j] = t.r[(KS + j) % kPAR];
    }
    // Schedule: the ring's first reads (when loaded here), then per K-step its MFMA and the LDS
    // read that refills the slot it freed, so that kPAR - 1 MFMAs cover each read's latency.
    // Left to itself the compiler sinks every read to just before its MFMA (two reads, a wait
    // for both, two MFMAs), exposing the LDS latency at every other step.
    if constexpr (kLoadFirst) __builtin_amdgcn_sched_group_barrier(0x100, kPAR, 0);   // LDS read
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
        if (ks + kPAR < KS || kNext) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
}

__device__ inline const lds_u8 *pstage(lds_u8 *ring, int64_t g) { return ring + (int)((uint32_t)g % kPStages) * kPStageBytes; }

// A pair of phases (the two halves of one M-block's contraction) between barriers; the
// accumulation starts from `init` (the M-block's float32 biases, or zero).
__device__ __attribute__((always_inline)) inline void paper_pair(PRing &rg, lds_u8 *ring, PAR &ar,
                                                                 const bf16x8 (&bin)[kPNKB][1], f32x16 &acc,
                                                                 const f32x16 &init, int wave, int lane) {
    acc = init;
    paper_fetch_next(rg, ring, wave, lane);
    pchain<16, 0, true, true>(pstage(ring, rg.g), pstage(ring, rg.g + 1), ar, bin, acc, lane);
    ++rg.g;
    paper_fetch_next(rg, ring, wave, lane);
    pchain<16, 16, false, false>(pstage(ring, rg.g), nullptr, ar, bin, acc, lane);
    ++rg.g;
    paper_stage_wait();
    __syncthreads();
}

// Compile-time loop: f(integral_constant<I>) for I = I0 .. N - 1, so that register arrays are
// indexed by constants however large the body (a 16-step loop over 33-MFMA phases is beyond
// what the unroller takes on by itself).
template <int I, int N, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ __attribute__((always_inline)) inline uint32_t tile_mask(const f32x16 &y) {
    uint32_t bits = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) bits |= (y[j] > 0.f ? 1u : 0u) << j;
    return bits;
}

// Masked adjoint tile -> bf16 B operands (K-blocks 2 mb, 2 mb + 1).
__device__ __attribute__((always_inline)) inline void pmasked_to_bf16(const f32x16 &y, uint32_t bits, int mb, bf16x8 (&b)[kPNKB][1]) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = __uint_as_float(__float_as_uint(y[j]) & (uint32_t)__builtin_amdgcn_sbfe((int)bits, j, 1));
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < 8; ++s) b[2 * mb + c][0][s] = (__bf16)v[8 * c + s];
}

// The 16 float32 biases of the rows this lane holds in M-block mb (rows 8 g + 4 h + i).
__device__ __attribute__((always_inline)) inline f32x16 pbias_tile(const float *bias, int mb, int h) {
    f32x16 v;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const f32x4 b4 = *reinterpret_cast<const f32x4 *>(bias + mb * 32 + 8 * g + 4 * h);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * g + i] = b4[i];
    }
    return v;
}

// Hidden layer l: bin -> bout (ReLU, bf16); masks of layer l to LDS for gradients.
template <bool kGrad>
__device__ __attribute__((always_inline)) inline void paper_fwd_layer(PRing &rg, lds_u8 *ring, PAR &ar, int l,
                                                                      const bf16x8 (&bin)[kPNKB][1],
                                                                      bf16x8 (&bout)[kPNKB][1], uint16_t *wmask,
                                                                      const float *s_bias, int wave, int lane, int h) {
    f32x16 acc[2];
    const float *lb = s_bias + (l - 1) * kPW;
    static_for<0, kPNMB>([&](auto mbc) __attribute__((always_inline)) {
        constexpr int mb = decltype(mbc)::value;
        paper_pair(rg, ring, ar, bin, acc[mb & 1], pbias_tile(lb, mb, h), wave, lane);
        if constexpr (mb > 0) {
            if (kGrad) wmask[(l * kPNMB + mb - 1) * 64 + lane] = (uint16_t)tile_mask(acc[(mb - 1) & 1]);
            relu_tile_to_bf16(acc[(mb - 1) & 1], mb - 1, 0, bout);
            asm volatile("" : "+v"(bout[2 * (mb - 1)][0]), "+v"(bout[2 * (mb - 1) + 1][0]));
        }
    });
    if (kGrad) wmask[(l * kPNMB + kPNMB - 1) * 64 + lane] = (uint16_t)tile_mask(acc[(kPNMB - 1) & 1]);
    relu_tile_to_bf16(acc[(kPNMB - 1) & 1], kPNMB - 1, 0, bout);
}

// Transposed hidden layer l: adjoint operands of layer l's outputs -> masked adjoint operands
// of layer l - 1's outputs.
__device__ __attribute__((always_inline)) inline void paper_bwd_layer(PRing &rg, lds_u8 *ring, PAR &ar, int l,
                                                                      const bf16x8 (&bin)[kPNKB][1],
                                                                      bf16x8 (&bout)[kPNKB][1], const uint16_t *wmask,
                                                                      int wave, int lane) {
    f32x16 acc[2];
    static_for<0, kPNMB>([&](auto mbc) __attribute__((always_inline)) {
        constexpr int mb = decltype(mbc)::value;
        paper_pair(rg, ring, ar, bin, acc[mb & 1], f32x16{}, wave, lane);
        if constexpr (mb > 0) {
            pmasked_to_bf16(acc[(mb - 1) & 1], wmask[((l - 1) * kPNMB + mb - 1) * 64 + lane], mb - 1, bout);
            asm volatile("" : "+v"(bout[2 * (mb - 1)][0]), "+v"(bout[2 * (mb - 1) + 1][0]));
        }
    });
    pmasked_to_bf16(acc[(kPNMB - 1) & 1], wmask[((l - 1) * kPNMB + kPNMB - 1) * 64 + lane], kPNMB - 1, bout);
}

struct PaperArgs {
    const uint8_t *blob;
    int depth;
    const float *rays;     // [5][n]
    int64_t n;
    const float *g_dist;   // seeds (NULL = 0)
    float *dist_out;       // or NULL
    float *g_rays;         // [5][n] or NULL
};

template <bool kGrad>
__global__ __launch_bounds__(kPWaves * 64, 1) void paper_stream_kernel(PaperArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int depth = a.depth;
    const int64_t n = a.n;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5, col = lane & 31;
    const PaperLayout L = paper_layout(depth, kBF16);
    const PLds S = paper_lds(depth, kGrad);
    lds_u8 *ring = (lds_u8 *)(smem + S.ring);
    const float *s_l0 = reinterpret_cast<const float *>(smem + S.l0);
    const float *s_row = reinterpret_cast<const float *>(smem + S.row);
    const float *s_bias = reinterpret_cast<const float *>(smem + S.bias);
    uint16_t *wmask = reinterpret_cast<uint16_t *>(smem + S.mask) + wave * depth * kPNMB * 64;

    const int64_t ntile = (n + kPRays - 1) / kPRays;
    if ((int64_t)blockIdx.x >= ntile) return;   // the whole workgroup
    PRing rg;
    rg.blob = __builtin_amdgcn_make_buffer_rsrc((void *)a.blob, 0, (int)L.bytes, 0x00020000);
    rg.L = L;
    rg.np = 2 * kPNMB * (depth - 1) + 2 + (kGrad ? 2 * kPNMB * (depth - 1) + 2 : 0);
    rg.gend = ((ntile - blockIdx.x + gridDim.x - 1) / gridDim.x) * rg.np;
    rg.g = 0;
    rg.qf = 2 % rg.np;
    {   // first-layer tiles and the output row stay in LDS; phases 0 and 1 into stages 0 and 1
        const i32x4 *src = reinterpret_cast<const i32x4 *>(a.blob + L.l0_off);
        for (int i = threadIdx.x; i < kPNMB * kPK0 * 16; i += blockDim.x)
            reinterpret_cast<i32x4 *>(smem + S.l0)[i] = src[i];
        const float *row = reinterpret_cast<const float *>(a.blob + L.row_off);
        for (int i = threadIdx.x; i < kPW + 4; i += blockDim.x) reinterpret_cast<float *>(smem + S.row)[i] = row[i];
        const float *bias = reinterpret_cast<const float *>(a.blob + L.bias_off);
        for (int i = threadIdx.x; i < (depth - 1) * kPW; i += blockDim.x) reinterpret_cast<float *>(smem + S.bias)[i] = bias[i];
        paper_fetch(rg, 0, 0, ring, wave, lane);
        paper_fetch(rg, 1, 1 % rg.np, ring, wave, lane);
        paper_stage_wait();
        __syncthreads();
    }
    const float out_bias = s_row[kPW];

    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int64_t r = t * kPRays + wave * 32 + col;
        const bool valid = r < n;
        float v[kInRaw];
#pragma unroll
        for (int j = 0; j < kInRaw; ++j) v[j] = valid ? a.rays[(int64_t)j * n + r] : 0.f;
        const bool nan_ray = isnan(v[0]) || isnan(v[1]) || isnan(v[2]) || isnan(v[3]) || isnan(v[4]);
        bf16x8 b0[kPNKB][1], b1[kPNKB][1];
        // ---- first layer: float32 MFMA over (x, y), (z, theta), (phi, 1), ReLU -> bf16 into b0
        {
            const float in0 = h ? v[1] : v[0], in1 = h ? v[3] : v[2], in2 = h ? 1.f : v[4];
#pragma unroll
            for (int mb = 0; mb < kPNMB; ++mb) {
                f32x16 acc = f32x16{};
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(s_l0[(mb * kPK0 + 0) * 64 + lane], in0, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(s_l0[(mb * kPK0 + 1) * 64 + lane], in1, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(s_l0[(mb * kPK0 + 2) * 64 + lane], in2, acc, 0, 0, 0);
                if (kGrad) wmask[mb * 64 + lane] = (uint16_t)tile_mask(acc);
                relu_tile_to_bf16(acc, mb, 0, b0);
            }
        }
        PAR ar;
        // ---- hidden layers alternating b0 -> b1 -> b0 ...; the last output ends in b0
        int l = 1;
        if ((depth - 1) % 2 == 1) {
            paper_fwd_layer<kGrad>(rg, ring, ar, 1, b0, b1, wmask, s_bias, wave, lane, h);
#pragma unroll
            for (int kb = 0; kb < kPNKB; ++kb) b0[kb][0] = b1[kb][0];
            l = 2;
        }
        for (; l + 1 < depth; l += 2) {
            paper_fwd_layer<kGrad>(rg, ring, ar, l, b0, b1, wmask, s_bias, wave, lane, h);
            paper_fwd_layer<kGrad>(rg, ring, ar, l + 1, b1, b0, wmask, s_bias, wave, lane, h);
        }
        // ---- output: rows 0 (the bf16 row) and 1 (its remainder) of lane half 0
        f32x16 hacc;
        paper_pair(rg, ring, ar, b0, hacc, f32x16{}, wave, lane);
        {
            const float d = __shfl(hacc[0] + hacc[1], col) + out_bias;
            if (h == 0 && valid && a.dist_out) a.dist_out[r] = nan_ray ? NAN : d;
        }
        if constexpr (kGrad) {
            const float gd = (valid && a.g_dist) ? a.g_dist[r] : 0.f;
            // ---- adjoint of the last hidden layer: output row x seed, masked -> b0
#pragma unroll
            for (int mb = 0; mb < kPNMB; ++mb) {
                f32x16 y;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const f32x4 w4 = *reinterpret_cast<const f32x4 *>(s_row + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                    for (int i = 0; i < 4; ++i) y[4 * g + i] = w4[i] * gd;
                }
                pmasked_to_bf16(y, wmask[((depth - 1) * kPNMB + mb) * 64 + lane], mb, b0);
            }
            // ---- transposed hidden layers from the top; the last adjoint ends in b0
            int lb = depth - 1;
            if (lb % 2 == 1) {
                paper_bwd_layer(rg, ring, ar, lb, b0, b1, wmask, wave, lane);
#pragma unroll
                for (int kb = 0; kb < kPNKB; ++kb) b0[kb][0] = b1[kb][0];
                --lb;
            }
            for (; lb >= 2; lb -= 2) {
                paper_bwd_layer(rg, ring, ar, lb, b0, b1, wmask, wave, lane);
                paper_bwd_layer(rg, ring, ar, lb - 1, b1, b0, wmask, wave, lane);
            }
            // ---- transposed first layer: rows 0..4 = d/d(ox, oy, oz, theta, phi)
            f32x16 gacc;
            paper_pair(rg, ring, ar, b0, gacc, f32x16{}, wave, lane);
            // row 8 (j / 4) + 4 h + j % 4: rows 0..3 in lane half 0 (j = 0..3), row 4 in half 1 (j = 0)
            if (valid && a.g_rays) {
                if (h == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) a.g_rays[(int64_t)j * n + r] = nan_ray ? NAN : gacc[j];
                } else {
                    a.g_rays[(int64_t)4 * n + r] = nan_ray ? NAN : gacc[0];
                }
            }
        }
    }
}


// ------------------------------------------------------------------------------ float32 sweep
// Float32 queries, input gradients and the training sweep (paper_sweep_kernel): a workgroup
// of eight waves takes 32 rays at a time and keeps their layer values in LDS ([ray][unit],
// row pitch 516 floats); every wave reads a layer's whole input from LDS as B operands of the
// 32x32x2 float32 MFMA (four K-steps per 16-byte read) and produces two of the 16 M-blocks;
// weight tiles come from the L2-resident blob (one 256-byte tile per wave, M-block and K-step,
// four groups of four K-steps in flight).  The output row and the transposed first layer (one
// M-block each) split their 256 K-steps over the eight waves and add the partial sums in wave
// order.  ReLU masks stay in LDS for the reverse sweep; the training sweep also writes every
// layer's activations and adjoints for the weight-gradient products.
constexpr int kSW = 8;            // waves
constexpr int kSR = 32;           // rays per tile
constexpr int kSXP = kPW + 4;     // row pitch of the layer values (floats)

struct SLds {
    int x, x0, mask, part, seed, loss, bytes;
};
__host__ __device__ inline SLds sweep_lds(int depth) {
    SLds s;
    s.x = 0;
    s.x0 = s.x + kSR * kSXP * 4;
    s.mask = s.x0 + kSR * 8 * 4;
    s.part = s.mask + depth * kPNMB * 64 * 2;
    s.seed = s.part + kSW * 8 * 32 * 4;
    s.loss = s.seed + kSR * 4;
    s.bytes = s.loss + kSW * 4;
    return s;
}

struct SweepArgs {
    const uint8_t *blob;   // float32 blob
    int depth;
    const float *rays;     // [5][n]
    int64_t n;
    const float *g_dist;   // seeds (NULL: from the loss, or zero)
    const float *t_label;  // training: labels (+inf = miss); the seeds come from `loss`
    LossSpec loss;
    float inv_n;           // 1 / (loss normalisation)
    float *dist_out;       // or NULL
    float *g_rays;         // [5][n] or NULL
    float *ws_h;           // [depth][512][n] activations (training), or NULL
    float *ws_delta;       // [depth][512][n] adjoints, then [n] output seeds (training), or NULL
    float *loss_partial;   // [gridDim.x] (training)
    bool forward_only;
    // training dropout (inverted): unit u of ray r in hidden layer l is kept when the top 24
    // bits of H(K_l ^ (u << 32 | r)) are >= drop_thr, K_l = H(H(H(drop_seed) ^ drop_step) ^ l),
    // H the first output of SplitMix64 from a given state; kept units are scaled by drop_scale.
    // drop_thr = 0: no dropout (drop_scale is then ignored).
    uint32_t drop_thr;
    float drop_scale;
    uint64_t drop_seed;
    int64_t drop_step;
};

// H(x): the first output of a SplitMix64 generator (Steele, Lea and Flood, 2014) whose state
// is x: the state advances by the golden-ratio increment and the output function mixes it.
__host__ __device__ inline uint64_t splitmix_h(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Dropout keep bits of a lane's D-layout tile (units mb * 32 + 8 (q / 4) + 4 h + q % 4 of ray r).
__device__ inline uint32_t pdrop_bits(uint64_t key, uint32_t thr, int mb, int h, int64_t r) {
    uint32_t bits = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint64_t u = (uint64_t)(mb * 32 + 8 * (q / 4) + 4 * h + (q % 4));
        const uint64_t k = splitmix_h(key ^ ((u << 32) | (uint64_t)(uint32_t)r));
        bits |= ((uint32_t)(k >> 40) >= thr ? 1u : 0u) << q;
    }
    return bits;
}

// acc[j] (M-block j of this wave's NM, tiles j * 64 floats apart) += sum over KS K-steps from
// kb0 of tile (kb) x layer values X[ray][unit(kb, h)]; tiles: the first tile of K-step 0,
// kstride floats between K-steps.
template <int NM, int KS>
__device__ __attribute__((always_inline)) inline void psweep_mfma(const float *__restrict__ tiles, int kstride, int kb0,
                                                                  const float *X, int lane, f32x16 (&acc)[NM]) {
    const int h = lane >> 5, col = lane & 31;
    const float *t = tiles + lane + (int64_t)kb0 * kstride;
    constexpr int kG = 4;   // groups of four K-steps of weight tiles in flight
    float a[kG][NM][4];
#pragma unroll
    for (int g = 0; g < kG - 1; ++g)
#pragma unroll
        for (int j = 0; j < NM; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[g][j][q] = 4 * g < KS ? t[(int64_t)(4 * g + q) * kstride + j * 64] : 0.f;
#pragma unroll 2
    for (int kb = 0; kb < KS; kb += 4) {
        if (kb + 4 * (kG - 1) < KS) {
#pragma unroll
            for (int j = 0; j < NM; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) a[kG - 1][j][q] = t[(int64_t)(kb + 4 * (kG - 1) + q) * kstride + j * 64];
        }
        const int k = kb0 + kb;
        const f32x4 b4 = *reinterpret_cast<const f32x4 *>(X + col * kSXP + 32 * (k / 16) + 8 * ((k % 16) / 4) + 4 * h);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < NM; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][j][q], b4[q], acc[j], 0, 0, 0);
#pragma unroll
        for (int g = 0; g + 1 < kG; ++g)
#pragma unroll
            for (int j = 0; j < NM; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) a[g][j][q] = a[g + 1][j][q];
    }
}

// Stores value j of a lane's D-layout tile (unit mb * 32 + 8 (j / 4) + 4 h + j % 4 of ray col)
// into the layer values and, when given, into a [512][n] side output.
__device__ __attribute__((always_inline)) inline void pstore_tile(const float (&y)[16], int mb, int h, int col, float *X,
                                                                  float *side, int64_t n, int64_t r, bool valid) {
#pragma unroll
    for (int g = 0; g < 4; ++g)
        *reinterpret_cast<f32x4 *>(X + col * kSXP + mb * 32 + 8 * g + 4 * h) = f32x4{y[4 * g], y[4 * g + 1], y[4 * g + 2], y[4 * g + 3]};
    if (side && valid) {
        float *dst = side + (int64_t)(mb * 32 + 4 * h) * n + r;
#pragma unroll
        for (int j = 0; j < 16; ++j) dst[(int64_t)(8 * (j / 4) + (j % 4)) * n] = y[j];
    }
}

__global__ __launch_bounds__(kSW * 64, 1) void paper_sweep_kernel(SweepArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int depth = a.depth;
    const int64_t n = a.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, col = lane & 31;
    const int mb0 = 2 * wave;   // this wave's M-blocks mb0, mb0 + 1
    const SLds S = sweep_lds(depth);
    float *X = reinterpret_cast<float *>(smem + S.x);
    float *X0 = reinterpret_cast<float *>(smem + S.x0);
    uint16_t *s_mask = reinterpret_cast<uint16_t *>(smem + S.mask);
    float *s_part = reinterpret_cast<float *>(smem + S.part);
    float *s_seed = reinterpret_cast<float *>(smem + S.seed);
    float *s_loss = reinterpret_cast<float *>(smem + S.loss);
    const PaperLayout L = paper_layout(depth, kFP32);
    const float *l0 = reinterpret_cast<const float *>(a.blob + L.l0_off);
    const float *hid = reinterpret_cast<const float *>(a.blob + L.hid_off);
    const float *head = reinterpret_cast<const float *>(a.blob + L.head_off);
    const float *tr = reinterpret_cast<const float *>(a.blob + L.tr_off);
    const float *bias = reinterpret_cast<const float *>(a.blob + L.bias_off);
    const float *row = reinterpret_cast<const float *>(a.blob + L.row_off);
    const bool train = a.ws_h != nullptr;
    const bool drop = a.drop_thr != 0;
    const float dscale = drop ? a.drop_scale : 1.f;   // 1 (exact) without dropout
    const uint64_t drop_base = splitmix_h(splitmix_h(a.drop_seed) ^ (uint64_t)a.drop_step);
    auto layer_key = [&](int l) { return splitmix_h(drop_base ^ (uint64_t)l); };
    float loss_acc = 0.f;
    auto mask_at = [&](int l, int mb) -> uint16_t & { return s_mask[(l * kPNMB + mb) * 64 + lane]; };

    const int64_t ntile = (n + kSR - 1) / kSR;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t r = tile * kSR + col;
        const bool valid = r < n;
        // ---- the raw inputs (and 1 for the first layer's bias) of the tile's 32 rays
        if (threadIdx.x < kSR * 8) {
            const int ray = threadIdx.x / 8, k = threadIdx.x % 8;
            const int64_t rr = tile * kSR + ray;
            X0[ray * 8 + k] = k < kInRaw ? (rr < n ? a.rays[(int64_t)k * n + rr] : 0.f) : (k == kInRaw ? 1.f : 0.f);
        }
        __syncthreads();
        bool nan_ray = false;
#pragma unroll
        for (int k = 0; k < kInRaw; ++k) nan_ray |= isnan(X0[col * 8 + k]);
        // ---- first layer: three K-steps over (x, y), (z, theta), (phi, 1)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int mb = mb0 + j;
            f32x16 acc = f32x16{};
#pragma unroll
            for (int ks = 0; ks < kPK0; ++ks)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(l0[(mb * kPK0 + ks) * 64 + lane], X0[col * 8 + 2 * ks + h], acc, 0, 0, 0);
            float y[16];
            uint32_t bits = 0;
            const uint32_t keep = drop ? pdrop_bits(layer_key(0), a.drop_thr, mb, h, r) : 0xFFFFu;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const bool on = acc[q] > 0.f && ((keep >> q) & 1u);
                y[q] = on ? acc[q] * dscale : 0.f;
                bits |= (on ? 1u : 0u) << q;
            }
            mask_at(0, mb) = (uint16_t)bits;
            pstore_tile(y, mb, h, col, X, train ? a.ws_h : nullptr, n, r, valid);
        }
        __syncthreads();
        // ---- hidden layers: every wave reads the whole input, then writes its two M-blocks
        for (int l = 1; l < depth; ++l) {
            f32x16 acc[2] = {f32x16{}, f32x16{}};
            psweep_mfma<2, kPF32K>(hid + (int64_t)(l - 1) * kPF32K * kPNMB * 64 + mb0 * 64, kPNMB * 64, 0, X, lane, acc);
            __syncthreads();   // the input is read by every wave before anyone overwrites it
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int mb = mb0 + j;
                float y[16];
                uint32_t bits = 0;
                const uint32_t keep = drop ? pdrop_bits(layer_key(l), a.drop_thr, mb, h, r) : 0xFFFFu;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const f32x4 b4 = *reinterpret_cast<const f32x4 *>(bias + (l - 1) * kPW + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float z = acc[j][4 * g + i] + b4[i];
                        const bool on = z > 0.f && ((keep >> (4 * g + i)) & 1u);
                        y[4 * g + i] = on ? z * dscale : 0.f;
                        bits |= (on ? 1u : 0u) << (4 * g + i);
                    }
                }
                mask_at(l, mb) = (uint16_t)bits;
                pstore_tile(y, mb, h, col, X, train ? a.ws_h + (int64_t)l * kPW * n : nullptr, n, r, valid);
            }
            __syncthreads();
        }
        // ---- output row: 32 K-steps per wave, partial sums added in wave order
        {
            f32x16 hacc[1] = {f32x16{}};
            psweep_mfma<1, kPF32K / kSW>(head, 64, wave * (kPF32K / kSW), X, lane, hacc);
            if (h == 0) s_part[wave * 32 + col] = hacc[0][0];   // row 0
        }
        __syncthreads();
        if (wave == 0) {
            float d = 0.f;
#pragma unroll
            for (int w = 0; w < kSW; ++w) d += s_part[w * 32 + col];
            d += row[kPW];
            float gd = 0.f;
            if (a.t_label) {
                const float t = valid ? a.t_label[r] : INFINITY;
                float g0, g1;
                const float term = ray_loss(0.f, d, t, a.inv_n, 0.f, a.loss, g0, g1);
                gd = valid ? g1 : 0.f;
                if (h == 0 && valid) loss_acc += term;
            } else if (a.g_dist && valid) {
                gd = a.g_dist[r];
            }
            if (h == 0) {
                s_seed[col] = gd;
                if (valid && a.dist_out) a.dist_out[r] = nan_ray ? NAN : d;
                if (valid && train) a.ws_delta[(int64_t)depth * kPW * n + r] = gd;
            }
        }
        __syncthreads();
        if (a.forward_only) continue;
        // ---- adjoint of the last hidden layer: output row x seed, masked
        {
            const float gd = s_seed[col];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int mb = mb0 + j;
                const uint32_t bits = mask_at(depth - 1, mb);
                float y[16];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const f32x4 w4 = *reinterpret_cast<const f32x4 *>(row + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                    for (int i = 0; i < 4; ++i) y[4 * g + i] = ((bits >> (4 * g + i)) & 1u) ? w4[i] * gd * dscale : 0.f;
                }
                pstore_tile(y, mb, h, col, X, train ? a.ws_delta + (int64_t)(depth - 1) * kPW * n : nullptr, n, r, valid);
            }
        }
        __syncthreads();
        // ---- transposed hidden layers from the top: X holds layer l's adjoint
        for (int l = depth - 1; l >= 1; --l) {
            f32x16 acc[2] = {f32x16{}, f32x16{}};
            psweep_mfma<2, kPF32K>(tr + (int64_t)(l - 1) * kPF32K * kPNMB * 64 + mb0 * 64, kPNMB * 64, 0, X, lane, acc);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int mb = mb0 + j;
                const uint32_t bits = mask_at(l - 1, mb);
                float y[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) y[q] = ((bits >> q) & 1u) ? acc[j][q] * dscale : 0.f;
                pstore_tile(y, mb, h, col, X, train ? a.ws_delta + (int64_t)(l - 1) * kPW * n : nullptr, n, r, valid);
            }
            __syncthreads();
        }
        // ---- transposed first layer: rows 0..4 = d/d(ox, oy, oz, theta, phi)
        if (a.g_rays) {
            f32x16 gacc[1] = {f32x16{}};
            psweep_mfma<1, kPF32K / kSW>(tr + (int64_t)(depth - 1) * kPF32K * kPNMB * 64, 64, wave * (kPF32K / kSW), X,
                                         lane, gacc);
            // rows 0..3 in lane half 0 (values 0..3), row 4 in lane half 1 (value 0)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (h == 0) s_part[(wave * 8 + k) * 32 + col] = gacc[0][k];
            if (h == 1) s_part[(wave * 8 + 4) * 32 + col] = gacc[0][0];
            __syncthreads();
            if (wave == 0 && h == 0 && valid) {
#pragma unroll
                for (int k = 0; k < kInRaw; ++k) {
                    float g = 0.f;
#pragma unroll
                    for (int w = 0; w < kSW; ++w) g += s_part[(w * 8 + k) * 32 + col];
                    a.g_rays[(int64_t)k * n + r] = nan_ray ? NAN : g;
                }
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
        for (int w = 0; w < kSW; ++w) t += s_loss[w];
        a.loss_partial[blockIdx.x] = t;
    }
}

// Weight normalisation backward, one wave per hidden row i of layer l (u = v / |v|, G = dL/dW
// of the folded row): dL/dg = G . u, dL/dv = (g / |v|) (G - (G . u) u); the bias gradient is
// copied; the output row's gradient and bias gradient are copied as they are.
// gW: the plain gradients, per layer [512][in_l] then [512] (the output layer [512] then [1]).
__global__ void paper_wn_grad_kernel(const float *__restrict__ params, const FF *__restrict__ norm,
                                     const float *__restrict__ gW, int depth, float *__restrict__ g, bool accumulate) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (row > (int64_t)depth * kPW) return;
    if (row == (int64_t)depth * kPW) {   // the output layer: plain copy
        const int64_t po = paper_layer_off(depth), go = gw_layer_off(depth);
        for (int k = lane; k <= kPW; k += 64) g[po + k] = accumulate ? g[po + k] + gW[go + k] : gW[go + k];
        return;
    }
    const int l = (int)(row / kPW), i = (int)(row % kPW), in = paper_in(l);
    const int64_t po = paper_layer_off(l), go = gw_layer_off(l);
    const float *v = params + po + (int64_t)i * in;
    const float *G = gW + go + (int64_t)i * in;
    const float nv = norm[row].hi + norm[row].lo, gain = params[po + (int64_t)kPW * in + i];
    float dot = 0.f;
    for (int k = lane; k < in; k += 64) dot = fmaf(G[k], v[k], dot);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off);
    const float gg = dot / nv;   // G . u
    const float scale = gain / nv;
    float *gv = g + po + (int64_t)i * in;
    for (int k = lane; k < in; k += 64) {
        const float d = scale * (G[k] - gg * (v[k] / nv));
        gv[k] = accumulate ? gv[k] + d : d;
    }
    if (lane == 0) {
        float *gg_out = g + po + (int64_t)kPW * in + i, *gb_out = gg_out + kPW;
        const float db = gW[go + (int64_t)kPW * in + i];
        *gg_out = accumulate ? *gg_out + gg : gg;
        *gb_out = accumulate ? *gb_out + db : db;
    }
}

// Sum of the loss partials in a fixed order (one block).
__global__ void paper_sum_kernel(const float *__restrict__ part, int cnt, float *out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

int cu_count_paper();
int64_t paper_sweep_grid(int64_t n) {
    return std::max<int64_t>(1, std::min<int64_t>((n + kSR - 1) / kSR, (int64_t)cu_count_paper()));
}

int cu_count_paper() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    });
    return cus;
}

template <bool kGrad>
ddf_status launch_paper_stream(const PaperArgs &a, hipStream_t s) {
    auto kern = paper_stream_kernel<kGrad>;
    static std::once_flag once;
    std::call_once(once, [&] { (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kPLds); });
    const size_t lds = paper_lds(a.depth, kGrad).bytes;
    const int64_t ntile = (a.n + kPRays - 1) / kPRays;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ntile, cu_count_paper()));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kPWaves * 64), lds, s, a);
    return launch_status("ddf paper network kernel");
}

ddf_status launch_paper_sweep(const SweepArgs &a, hipStream_t s) {
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void *)paper_sweep_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kPLds);
    });
    const size_t lds = sweep_lds(a.depth).bytes;
    hipLaunchKernelGGL(paper_sweep_kernel, dim3((unsigned)paper_sweep_grid(a.n)), dim3(kSW * 64), lds, s, a);
    return launch_status("ddf paper network float32 sweep");
}

// Workspace of the float32 parameter gradient for n rays.
struct PaperWs {
    float *h, *delta, *gw, *part, *dbpart, *loss_part;
    size_t bytes;
};
inline size_t pal256(size_t x) { return (x + 255) & ~(size_t)255; }
PaperWs paper_ws(int depth, int64_t n, void *base) {
    PaperWs w{};
    uint8_t *p = reinterpret_cast<uint8_t *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        float *q = p ? reinterpret_cast<float *>(p + off) : nullptr;
        off += pal256(bytes);
        return q;
    };
    size_t part = 0, db = 0;
    for (int l = 0; l <= depth; ++l) {
        const int M = l == depth ? 1 : kPW, N = l == 0 ? kInRaw : kPW;
        part = std::max(part, dw_partial_floats(M, N, n));
        db = std::max(db, (size_t)((n + dw_chunk(M, N) - 1) / dw_chunk(M, N)) * M);
    }
    w.h = take((size_t)depth * kPW * n * 4);
    w.delta = take(((size_t)depth * kPW + 1) * n * 4);
    w.gw = take((size_t)gw_floats(depth) * 4);
    w.part = take(part * 4);
    w.dbpart = take(db * 4);
    w.loss_part = take(4096 * 4);
    w.bytes = off;
    return w;
}

// Float32 parameter gradient of n rays: the training sweep (seeds from g_dist, or from the loss
// when t_label is given), the weight-gradient products, the weight-normalisation backward.
ddf_status paper_param_grad(const ddf_paper_net *net, const float *params, const float *rays, int64_t n,
                            const float *g_dist, const float *t_label, LossSpec loss, float *g_rays, float *g_params,
                            bool accumulate, const PaperWs &w, hipStream_t s, uint32_t drop_thr = 0,
                            float drop_scale = 1.f, uint64_t drop_seed = 0, int64_t drop_step = 0) {
    const int depth = net->depth;
    SweepArgs a{};
    a.drop_thr = drop_thr;
    a.drop_scale = drop_scale;
    a.drop_seed = drop_seed;
    a.drop_step = drop_step;
    a.blob = (const uint8_t *)net->packed;
    a.depth = depth;
    a.rays = rays;
    a.n = n;
    a.g_dist = g_dist;
    a.t_label = t_label;
    a.loss = loss;
    a.inv_n = 1.0f / (float)n;
    a.g_rays = g_rays;
    a.ws_h = w.h;
    a.ws_delta = w.delta;
    a.loss_partial = w.loss_part;
    if (ddf_status st = launch_paper_sweep(a, s)) return st;
    for (int l = 0; l <= depth; ++l) {
        const int M = l == depth ? 1 : kPW, N = l == 0 ? kInRaw : kPW;
        const float *A = w.delta + (int64_t)l * kPW * n;   // the output seeds follow the last adjoint
        const float *B = l == 0 ? rays : w.h + (int64_t)(l - 1) * kPW * n;
        if (ddf_status st = dw_product(A, B, M, N, n, w.part, w.dbpart, w.gw + gw_layer_off(l), false, s)) return st;
    }
    const PaperLayout L = paper_layout(depth, kFP32);
    const FF *norm = reinterpret_cast<const FF *>(reinterpret_cast<const uint8_t *>(net->packed) + L.bytes);
    const int rows = depth * kPW + 1;
    hipLaunchKernelGGL(paper_wn_grad_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, params, norm, (const float *)w.gw,
                       depth, g_params, accumulate);
    return launch_status("ddf paper network weight-norm gradient");
}

ddf_status check_paper(const ddf_paper_net *net, const char *who) {
    DDF_REQUIRE(net && net->packed, DDF_ERR_INVALID_ARG, "%s: NULL network", who);
    DDF_REQUIRE(net->depth >= 1 && net->depth <= kPMaxDepth, DDF_ERR_UNSUPPORTED, "%s: depth %d not supported (1..8)",
                who, net->depth);
    DDF_REQUIRE(net->precision == kFP32 || net->precision == kBF16, DDF_ERR_UNSUPPORTED,
                "%s: precision %d not supported (float32 or bf16)", who, net->precision);
    return DDF_OK;
}

}  // namespace
}  // namespace ddf

using namespace ddf;

extern "C" ddf_status ddf_paper_param_count(int32_t depth, int64_t *count) {
    DDF_REQUIRE(count, DDF_ERR_INVALID_ARG, "ddf_paper_param_count: NULL output");
    DDF_REQUIRE(depth >= 1 && depth <= kPMaxDepth, DDF_ERR_UNSUPPORTED, "ddf_paper_param_count: depth %d not supported (1..8)",
                depth);
    *count = paper_params(depth);
    return DDF_OK;
}

extern "C" ddf_status ddf_paper_packed_bytes(int32_t depth, int32_t precision, size_t *bytes) {
    DDF_REQUIRE(bytes, DDF_ERR_INVALID_ARG, "ddf_paper_packed_bytes: NULL output");
    DDF_REQUIRE(depth >= 1 && depth <= kPMaxDepth, DDF_ERR_UNSUPPORTED, "ddf_paper_packed_bytes: depth %d not supported (1..8)",
                depth);
    DDF_REQUIRE(precision == kFP32 || precision == kBF16, DDF_ERR_UNSUPPORTED,
                "ddf_paper_packed_bytes: precision %d not supported", precision);
    *bytes = (size_t)paper_layout(depth, precision).bytes + (size_t)depth * kPW * 8;   // + the row norms
    return DDF_OK;
}

extern "C" ddf_status ddf_paper_pack(const float *params, int32_t depth, int32_t precision, void *packed,
                                     ddf_stream stream) {
    DDF_REQUIRE(params && packed, DDF_ERR_INVALID_ARG, "ddf_paper_pack: NULL params or output");
    DDF_REQUIRE(depth >= 1 && depth <= kPMaxDepth, DDF_ERR_UNSUPPORTED, "ddf_paper_pack: depth %d not supported (1..8)", depth);
    DDF_REQUIRE(precision == kFP32 || precision == kBF16, DDF_ERR_UNSUPPORTED, "ddf_paper_pack: precision %d not supported",
                precision);
    hipStream_t s = as_stream(stream);
    const PaperLayout L = paper_layout(depth, precision);
    // the row scales g / |v| live after the blob proper
    FF *norm = reinterpret_cast<FF *>(reinterpret_cast<uint8_t *>(packed) + L.bytes);
    const int rows = depth * kPW;
    hipLaunchKernelGGL(paper_norm_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, params, depth, norm);
    if (ddf_status st = launch_status("ddf_paper_pack")) return st;
    hipLaunchKernelGGL(paper_pack_kernel, dim3(2048), dim3(256), 0, s, params, (const FF *)norm, depth, precision,
                       (uint8_t *)packed);
    return launch_status("ddf_paper_pack");
}

extern "C" ddf_status ddf_paper_forward(const ddf_paper_net *net, const float *rays, int64_t n, float *dist_out,
                                        ddf_stream stream) {
    if (ddf_status st = check_paper(net, "ddf_paper_forward")) return st;
    DDF_REQUIRE(n >= 0, DDF_ERR_INVALID_ARG, "ddf_paper_forward: negative n");
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(rays && dist_out, DDF_ERR_INVALID_ARG, "ddf_paper_forward: NULL array");
    if (net->precision == kFP32) {
        SweepArgs a{};
        a.blob = (const uint8_t *)net->packed;
        a.depth = net->depth;
        a.rays = rays;
        a.n = n;
        a.dist_out = dist_out;
        a.forward_only = true;
        return launch_paper_sweep(a, as_stream(stream));
    }
    PaperArgs a{};
    a.blob = (const uint8_t *)net->packed;
    a.depth = net->depth;
    a.rays = rays;
    a.n = n;
    a.dist_out = dist_out;
    return launch_paper_stream<false>(a, as_stream(stream));
}

extern "C" ddf_status ddf_paper_workspace_size(int32_t depth, int64_t n, size_t *bytes) {
    DDF_REQUIRE(bytes && n >= 0, DDF_ERR_INVALID_ARG, "ddf_paper_workspace_size: bad argument");
    DDF_REQUIRE(depth >= 1 && depth <= kPMaxDepth, DDF_ERR_UNSUPPORTED, "ddf_paper_workspace_size: depth %d not supported (1..8)",
                depth);
    *bytes = paper_ws(depth, n, nullptr).bytes;
    return DDF_OK;
}

extern "C" ddf_status ddf_paper_backward(const ddf_paper_net *net, const float *params, const float *rays, int64_t n,
                                         const float *g_dist, float *g_rays, float *g_params, uint32_t flags, void *ws,
                                         size_t ws_bytes, ddf_stream stream) {
    if (ddf_status st = check_paper(net, "ddf_paper_backward")) return st;
    DDF_REQUIRE(n >= 0, DDF_ERR_INVALID_ARG, "ddf_paper_backward: negative n");
    DDF_REQUIRE((flags & ~1u) == 0, DDF_ERR_INVALID_ARG, "ddf_paper_backward: unknown flags 0x%x", flags);
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(rays && (g_rays || g_params), DDF_ERR_INVALID_ARG, "ddf_paper_backward: nothing to compute");
    hipStream_t s = as_stream(stream);
    if (g_params) {
        DDF_REQUIRE(net->precision == kFP32, DDF_ERR_UNSUPPORTED,
                    "ddf_paper_backward: parameter gradients need a float32 network");
        DDF_REQUIRE(params, DDF_ERR_INVALID_ARG, "ddf_paper_backward: parameter gradients need the parameters");
        const PaperWs need = paper_ws(net->depth, n, nullptr);
        DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE, "ddf_paper_backward: workspace of %zu bytes needed",
                    need.bytes);
        return paper_param_grad(net, params, rays, n, g_dist, nullptr, LossSpec{0, 0.f}, g_rays, g_params,
                                (flags & 1u) != 0, paper_ws(net->depth, n, ws), s);
    }
    if (net->precision == kFP32) {
        SweepArgs a{};
        a.blob = (const uint8_t *)net->packed;
        a.depth = net->depth;
        a.rays = rays;
        a.n = n;
        a.g_dist = g_dist;
        a.g_rays = g_rays;
        return launch_paper_sweep(a, s);
    }
    PaperArgs a{};
    a.blob = (const uint8_t *)net->packed;
    a.depth = net->depth;
    a.rays = rays;
    a.n = n;
    a.g_dist = g_dist;
    a.g_rays = g_rays;
    return launch_paper_stream<true>(a, s);
}

extern "C" ddf_status ddf_paper_train_step(const ddf_paper_net *net, float *params, float *adam_m, float *adam_v,
                                           int64_t step, float lr, const float *rays, const float *t_label, int64_t n,
                                           const ddf_loss *loss, float dropout, uint64_t dropout_seed, float *loss_out,
                                           float *g_params, void *ws, size_t ws_bytes, ddf_stream stream) {
    if (ddf_status st = check_paper(net, "ddf_paper_train_step")) return st;
    DDF_REQUIRE(net->precision == kFP32, DDF_ERR_UNSUPPORTED, "ddf_paper_train_step: needs a float32 network");
    DDF_REQUIRE(n > 0 && params && adam_m && adam_v && rays && t_label && loss_out && g_params && step >= 1,
                DDF_ERR_INVALID_ARG, "ddf_paper_train_step: bad argument");
    DDF_REQUIRE(loss && (loss->kind == DDF_LOSS_CLAMP || loss->kind == DDF_LOSS_SQUISH), DDF_ERR_INVALID_ARG,
                "ddf_paper_train_step: the loss must be the clamp (Eq. 7) or the squish (Eq. 6) loss");
    DDF_REQUIRE(loss->kind != DDF_LOSS_CLAMP || (std::isfinite(loss->delta) && loss->delta > 0.f), DDF_ERR_INVALID_ARG,
                "ddf_paper_train_step: the clamp loss needs a finite delta > 0");
    DDF_REQUIRE(dropout >= 0.f && dropout < 1.f, DDF_ERR_INVALID_ARG, "ddf_paper_train_step: dropout must lie in [0, 1)");
    // kept when the draw's top 24 bits k satisfy k / 2^24 >= p, i.e. k >= ceil(p 2^24)
    const uint32_t thr = (uint32_t)std::ceil((double)dropout * 16777216.0);
    const float scale = thr ? (float)(1.0 / (1.0 - (double)dropout)) : 1.f;
    const PaperWs need = paper_ws(net->depth, n, nullptr);
    DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE, "ddf_paper_train_step: workspace of %zu bytes needed",
                need.bytes);
    hipStream_t s = as_stream(stream);
    const PaperWs w = paper_ws(net->depth, n, ws);
    if (ddf_status st = paper_param_grad(net, params, rays, n, nullptr, t_label, LossSpec{loss->kind, loss->delta},
                                         nullptr, g_params, false, w, s, thr, scale, dropout_seed, step))
        return st;
    hipLaunchKernelGGL(paper_sum_kernel, dim3(1), dim3(256), 0, s, (const float *)w.loss_part,
                       (int)paper_sweep_grid(n), loss_out);
    if (ddf_status st = launch_status("ddf_paper_train_step")) return st;
    if (ddf_status st = ddf_adam_step(params, g_params, adam_m, adam_v, paper_params(net->depth), step, lr, 0.9f, 0.999f,
                                      1e-8f, stream))
        return st;
    return ddf_paper_pack(params, net->depth, kFP32, const_cast<void *>(net->packed), stream);
}
