// Batched network query (Sec. IV-A: the field phi(x, theta) stored as MLP_w and
// evaluated for many oriented points at once) on CDNA4 matrix cores.
//
// One kernel evaluates the whole network per wave of rays: the Fourier encoding is
// computed in registers, every affine layer is a chain of 32x32 MFMAs whose result
// stays in the accumulators, and the epilogue (bias, ReLU, conversion to the next
// layer's operand type) writes straight into the next layer's B operands.  Only the
// 20 input bytes and 8 output bytes per ray touch HBM.  Weights are read as A operands
// from LDS (when the whole packed network fits in the 160 KiB of a CU) or from the
// L2-resident blob otherwise.  See mlp_layout.hpp for the operand numbering.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>

#include "common.hpp"
#include "mlp_device.hpp"
#include "mlp_layout.hpp"
#include "grad_args.hpp"
#include "rays_device.hpp"

namespace ddf {
namespace {

constexpr int kLdsBytes = 160 * 1024;

// ------------------------------------------------------------------------------ packing
// Weight of layer l (row m, input column c) from the flat parameter vector.
__device__ inline float weight_at(const float *params, int width, int depth, int l, int m, int c) {
    int64_t off = 0;
    int in = kInDim;
    for (int j = 0; j < l; ++j) {
        off += (int64_t)width * in + width;
        in = width;
    }
    const int out = l == depth ? 2 : width;
    (void)out;
    return params[off + (int64_t)m * in + c];
}

__device__ inline float bias_at(const float *params, int width, int depth, int l, int m) {
    int64_t off = 0;
    int in = kInDim;
    for (int j = 0; j <= l; ++j) {
        const int out = j == depth ? 2 : width;
        off += (int64_t)out * in;
        if (j < l) off += out;
        in = width;
    }
    return params[off + m];
}

// Value of A-operand slot s of `lane` in forward tile `tile` (layer, K-block, M-block decoded
// from the tile index), before conversion.
__device__ inline float forward_weight(const float *params, const NetLayout &L, int64_t tile, int lane, int s) {
    const int width = L.width, depth = L.depth, prec = L.prec;
    int l;
    int64_t t;
    if (tile < L.layer_tile(1) || depth == 0) {
        l = 0;
        t = tile;
    } else if (tile >= L.head_tile()) {
        l = depth;
        t = tile - L.head_tile();
    } else {
        l = 1 + (int)((tile - L.layer_tile(1)) / ((int64_t)(L.nkb + L.xkb) * L.nmb));
        t = tile - L.layer_tile(l);
    }
    const int nmb = l == depth ? 1 : L.nmb;
    const int kb = (int)(t / nmb), mb = (int)(t % nmb);
    const int h = lane / 32;
    const int m = mb * 32 + (lane % 32);
    if (l == depth && m >= 2) {
        // bf16 head: rows 2 and 3 carry what rounding rows 0 and 1 to bf16 left over (exact
        // in float32; rounded to bf16 when stored), so each output is the sum of two rows
        if (prec != kBF16 || m >= 4 || kb >= L.nkb) return 0.f;
        const float w = weight_at(params, width, depth, l, m - 2, prev_unit(prec, kb, h, s));
        return w - (float)(__bf16)w;
    }
    // bf16 bias split into hi + lo (see bias_kblocks)
    auto bias_part = [&](int part) {
        const float b = bias_at(params, width, depth, l, m);
        const float hi = (float)(__bf16)b;
        return part == 0 ? hi : (float)(__bf16)(b - hi);
    };
    if (l == 0) {
        const int f = layer0_feature(prec, kb, s);
        if (prec == kBF16 && h == 1 && (f == kBiasSlot0 || f == kBiasSlot1)) return bias_part(f == kBiasSlot0 ? 0 : 1);
        const int c = feature_column(h, f);
        return c >= 0 ? weight_at(params, width, depth, 0, m, c) : 0.f;
    }
    if (kb >= L.nkb) return (h == 0 && s < 2) ? bias_part(s) : 0.f;
    return weight_at(params, width, depth, l, m, prev_unit(prec, kb, h, s));
}

// Transposed tile of the input-gradient sweep: rows are the layer's inputs, K its outputs.
__device__ inline float grad_weight(const float *params, const NetLayout &L, int64_t tile, int lane, int s) {
    const int width = L.width, depth = L.depth, prec = L.prec;
    int l;
    int64_t t;
    if (tile < L.grad_layer_tile(1) || depth == 1) {
        l = 0;
        t = tile;
    } else {
        l = 1 + (int)((tile - L.grad_layer_tile(1)) / ((int64_t)L.nkb * L.nmb));
        t = tile - L.grad_layer_tile(l);
    }
    const int nmb = l == 0 ? kGradRowBlocks0 : L.nmb;
    const int kb = (int)(t / nmb), mb = (int)(t % nmb);
    const int m = mb * 32 + (lane % 32);
    const int k = prev_unit(prec, kb, lane / 32, s);   // an output unit of layer l
    if (l == 0) {
        const int c = feature_column(grad_row_half(m), grad_row_feature(m));
        return c >= 0 ? weight_at(params, width, depth, 0, k, c) : 0.f;
    }
    return weight_at(params, width, depth, l, k, m);
}

__device__ inline void store_slot(uint8_t *tile_base, int prec, int lane, int s, float w, float scale) {
    if (prec == kFP32) reinterpret_cast<float *>(tile_base)[lane] = w;
    else if (prec == kBF16) reinterpret_cast<uint16_t *>(tile_base)[lane * 8 + s] = bf16_bits(w);
    else tile_base[(s / 16) * 1024 + lane * 16 + s % 16] = fp8_bits(scale > 0.f ? w / scale : 0.f);   // load_a's halves
}

// One thread per packed element: forward tile slots, biases, scales, transposed tile
// slots, head rows.
__global__ void pack_kernel(const float *__restrict__ params, int width, int depth, int prec,
                            const float *__restrict__ scales, uint8_t *__restrict__ blob) {
    const NetLayout L = make_layout(width, depth, prec);
    const int slots = slots_per_lane(prec);
    const int64_t n_fwd = L.tiles * 64 * slots;
    const int64_t n_bias = (int64_t)width * depth + 4;
    const int64_t n_scale = 2 * (depth + 1);
    const int64_t n_grad = L.grad_tiles * 64 * slots;
    const int64_t n_head = prec == kFP8 ? 0 : 2 * (int64_t)width;
    const int64_t total = n_fwd + n_bias + n_scale + n_grad + n_head;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e;
        if (r < n_fwd) {
            const int s = (int)(r % slots), lane = (int)((r / slots) % 64);
            const int64_t tile = r / (slots * 64);
            int l = 0;
            if (prec == kFP8) {
                // the layer of this tile selects its weight scale
                l = tile < L.layer_tile(1) ? 0 : tile >= L.head_tile() ? depth
                    : 1 + (int)((tile - L.layer_tile(1)) / ((int64_t)(L.nkb + L.xkb) * L.nmb));
            }
            store_slot(blob + tile * tile_bytes(prec), prec, lane, s, forward_weight(params, L, tile, lane, s),
                       prec == kFP8 ? scales[2 * l] : 1.f);
            continue;
        }
        r -= n_fwd;
        if (r < n_bias) {
            float v = 0.f;
            const int l = (int)(r / width), m = (int)(r % width);
            if (l < depth) v = bias_at(params, width, depth, l, m);
            else if (r - (int64_t)width * depth < 2) v = bias_at(params, width, depth, depth, (int)(r - (int64_t)width * depth));
            reinterpret_cast<float *>(blob + L.bias_off)[r] = v;
            continue;
        }
        r -= n_bias;
        if (r < n_scale) {
            reinterpret_cast<float *>(blob + L.scale_off)[r] = scales ? scales[r] : 1.0f;
            continue;
        }
        r -= n_scale;
        if (r < n_grad) {
            const int s = (int)(r % slots), lane = (int)((r / slots) % 64);
            const int64_t tile = r / (slots * 64);
            store_slot(blob + L.grad_off + tile * tile_bytes(prec), prec, lane, s, grad_weight(params, L, tile, lane, s), 1.f);
            continue;
        }
        r -= n_grad;
        reinterpret_cast<float *>(blob + L.head_rows_off)[r] =
            weight_at(params, width, depth, depth, (int)(r / width), (int)(r % width));
    }
}

// Calibration: wave maximum of non-negative values, one atomic per wave (floats >= 0
// order as unsigned integers).
__device__ inline void wave_absmax(float v, unsigned int *dst) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) atomicMax(dst, __float_as_uint(v));
}

struct LdsConsts {
    float in_scale_inv;   // fp8: 1 / s_a of layer 0
    float alpha[9];       // fp8: s_w s_a / s_a(next) per layer; head: s_w s_a
    int aexp[9];          // fp8: alpha as an E8M0 exponent (127 + log2 alpha) for the MFMA scale
    int bad;              // fp8: some scale is not a positive power of two (outputs are NaN)
};

// fp8 epilogue of one accumulator tile: ReLU and the e4m3 range in one med3, then packed
// conversions (the conversion does not saturate, so the clamp must come first).
template <int NKB, int NB>
__device__ inline void fp8_tile_to_operands(const f32x16 &y, int mb, int nb, i32x8 (&b)[NKB][NB]) {
#pragma unroll
    for (int w4 = 0; w4 < 4; ++w4)
        b[mb / 2][nb][4 * (mb % 2) + w4] = pack_fp8x4(
            __builtin_amdgcn_fmed3f(y[4 * w4], 0.f, kFp8Max), __builtin_amdgcn_fmed3f(y[4 * w4 + 1], 0.f, kFp8Max),
            __builtin_amdgcn_fmed3f(y[4 * w4 + 2], 0.f, kFp8Max), __builtin_amdgcn_fmed3f(y[4 * w4 + 3], 0.f, kFp8Max));
}

__device__ inline f32x16 mfma_fp8_scaled(i32x8 a, i32x8 b, f32x16 c, int aexp) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, aexp, 0, 127);
}

// Bias values of the 16 accumulator rows a lane holds in M-block mb (rows 8 g + 4 h + i).
__device__ inline f32x16 bias_tile(const float *bias, int mb, int h) {
    f32x16 v;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const f32x4 b4 = *reinterpret_cast<const f32x4 *>(bias + mb * 32 + 8 * g + 4 * h);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * g + i] = b4[i];
    }
    return v;
}

// Scheduling groups of one step of dense_fp8 (constant arguments, hence the recursion).
template <int STEP, int NSTEP, int KIN, int NMB, int NB, int kAhead>
__device__ __attribute__((always_inline)) inline void fp8_schedule() {
    if constexpr (STEP < NSTEP) {
        constexpr int mb = STEP / KIN, ks = STEP % KIN;
        constexpr int nds = (STEP + kAhead < NSTEP ? 2 : 0) + (ks == 0 && mb + 1 < NMB ? 4 : 0);
        __builtin_amdgcn_sched_group_barrier(0x008, NB, 0);   // MFMA
        if constexpr (nds > 0) __builtin_amdgcn_sched_group_barrier(0x100, nds, 0);   // LDS read
        if constexpr (mb > 0) __builtin_amdgcn_sched_group_barrier(0x002, (24 * NB + KIN - 1) / KIN, 0);   // VALU
        fp8_schedule<STEP + 1, NSTEP, KIN, NMB, NB, kAhead>();
    }
}

// One fp8 affine layer with the weights in LDS, M-block outermost and software-pipelined
// like the bf16 layer.  The first MFMA of an M-block starts from the bias (stored in the
// next layer's activation units), the power-of-two rescale s_w s_a / s_next rides in the
// MFMA's A-operand scale, and the epilogue (one med3 and half a packed conversion per
// value) of block mb - 1 is interleaved with the MFMAs of block mb.
template <int W, int NB, int KIN>
__device__ __attribute__((always_inline)) inline void dense_fp8(const uint8_t *wsrc, int64_t t0,
                                                                const i32x8 (&bin)[W / 64][NB],
                                                                i32x8 (&bout)[W / 64][NB], const float *bias, int aexp,
                                                                int lane, int h) {
    constexpr int NMB = W / 32;
    constexpr int NSTEP = NMB * KIN;
    constexpr int kAhead = 2;
    auto tile_of = [&](int step) { return t0 + (int64_t)(step % KIN) * NMB + step / KIN; };
    __builtin_amdgcn_sched_barrier(0);   // nothing of this layer moves above its start
    i32x8 ring[kAhead];
#pragma unroll
    for (int i = 0; i < kAhead; ++i) ring[i] = load_a<kFP8>(wsrc, tile_of(i < NSTEP ? i : 0), lane);
    f32x16 acc[2][NB];   // M-blocks alternate between the two sets (no copies)
    f32x16 bnext = bias_tile(bias, 0, h);
#pragma unroll
    for (int step = 0; step < NSTEP; ++step) {
        const int mb = step / KIN, ks = step % KIN;
        const i32x8 a = ring[step % kAhead];
        if (step + kAhead < NSTEP) ring[step % kAhead] = load_a<kFP8>(wsrc, tile_of(step + kAhead), lane);
        f32x16 bv;
        if (ks == 0) {
            bv = bnext;
            if (mb + 1 < NMB) bnext = bias_tile(bias, mb + 1, h);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            acc[mb & 1][nb] = mfma_fp8_scaled(a, bin[ks][nb], ks == 0 ? bv : acc[mb & 1][nb], aexp);
        if (ks == KIN - 1) {
            if (mb > 0) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) fp8_tile_to_operands(acc[(mb - 1) & 1][nb], mb - 1, nb, bout);
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) fp8_tile_to_operands(acc[(NMB - 1) & 1][nb], NMB - 1, nb, bout);
    // Schedule: the ring and the first bias tile, then per step its MFMAs, its LDS refills
    // (A tile; the next M-block's bias at the first K-step) and a share of the previous
    // block's epilogue (24 VALU per ray block).  Without it the compiler issues every LDS
    // read of the layer first and runs out of registers.
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * kAhead + 4, 0);
    fp8_schedule<0, NSTEP, KIN, NMB, NB, kAhead>();
}

// Unsigned distance field epilogue (Eq. 5): the queries of one 32-ray block (lanes 0..31 hold
// ray r's logit z and distance d; lanes 32..63 pass valid = false) are point-major, query
// r = point * nd + direction.  Each hit becomes a 64-bit key (the distance's bits in an
// order-preserving form, then the direction index), lanes of one point take their minimum by
// a segmented suffix scan, and the first lane of each point meets the other blocks in one
// atomic minimum, so the smallest distance wins and, among equal ones, the lowest direction.
// A miss (z <= 0) and a NaN or +inf distance give no key.
// r / nd for 0 <= r < 2^31 without a division: with 2^(l-1) < nd <= 2^l and
// m = ceil(2^(31+l) / nd) (at most 32 bits), r / nd = (r m) >> (31 + l) exactly (the round-up
// method of Granlund and Montgomery, 1994).
struct UdfDiv {
    uint32_t m;
    int sh, nd;
};
__device__ inline UdfDiv udf_div_make(int nd) {
    const int l = nd > 1 ? 32 - __clz(nd - 1) : 0;
    return {(uint32_t)(((1ull << (31 + l)) + (uint64_t)nd - 1) / (uint64_t)nd), 31 + l, nd};
}
__device__ inline int udf_div(const UdfDiv &q, int r) { return (int)(((uint64_t)(uint32_t)r * q.m) >> q.sh); }

__device__ inline void udf_block_min(float z, float d, bool valid, int64_t r, const UdfDiv &q,
                                     unsigned long long *keys, int col) {
    const int nd = q.nd;
    const bool hit = valid && z > 0.f && d < INFINITY;
    const int p = valid ? udf_div(q, (int)r) : -1;
    const uint32_t u = __float_as_uint(d);
    const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    unsigned long long key = hit ? ((unsigned long long)ord << 32) | (uint32_t)((int)r - p * nd) : ~0ull;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const unsigned long long other = __shfl_down(key, off, 32);
        const int po = __shfl_down(p, off, 32);
        if (col + off < 32 && po == p && other < key) key = other;
    }
    const int prev = __shfl_up(p, 1, 32);
    if (p >= 0 && (col == 0 || prev != p) && key != ~0ull) atomicMin(keys + p, key);
}

// fp8 head with the weights in LDS: rows 0 (logit) and 1 (distance), bias as the start
// value, the power-of-two s_w s_a in the MFMA scale.  Lanes of half 0 hold both rows; the
// distance moves to half 1 so that every lane stores one value (no divergent branch near
// the matrix ops).
template <int W, int NB, bool kUdf = false>
__device__ __attribute__((always_inline)) inline void head_fp8(const uint8_t *wsrc, int64_t th,
                                                               const i32x8 (&bin)[W / 64][NB], const float *bias,
                                                               int aexp, bool bad, int lane, int h, int col,
                                                               int64_t base, int64_t n, const bool (&nan_ray)[NB],
                                                               float *logit_out, float *dist_out, UdfDiv udq = {},
                                                               unsigned long long *udf_keys = nullptr) {
    __builtin_amdgcn_sched_barrier(0);
    const f32x4 hb = *reinterpret_cast<const f32x4 *>(bias);   // logit, distance biases, 0, 0
    const float keep = (float)(1 - h);
    f32x16 c{};
    c[0] = hb[0] * keep;
    c[1] = hb[1] * keep;
    f32x16 acc[NB];
#pragma unroll
    for (int kb = 0; kb < W / 64; ++kb) {
        const i32x8 a = load_a<kFP8>(wsrc, th + kb, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma_fp8_scaled(a, bin[kb][nb], kb == 0 ? c : acc[nb], aexp);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const float d = __shfl(acc[nb][1], col);
        const int64_t r = base + nb * 32 + col;
        if constexpr (kUdf) {
            udf_block_min(acc[nb][0], d, h == 0 && r < n && !nan_ray[nb] && !bad, r, udq, udf_keys, col);
        } else {
            const float v = h ? d : acc[nb][0];
            float *dst = h ? dist_out : logit_out;
            if (r < n) dst[r] = (nan_ray[nb] || bad) ? NAN : v;
        }
    }
}

// MFMAs of one 32-row M-block of a layer for NB ray blocks (bf16 adds the bias K-block).
template <int P, int W, int NB, int KIN>
__device__ __attribute__((always_inline)) inline void mblock_mfma(const uint8_t *wsrc, int64_t t0, int mb,
                                                                  const typename OpOf<P>::T (&bin)[W / k_per_block(P)][NB],
                                                                  f32x16 (&acc)[NB], int lane, int h) {
    using Op = typename OpOf<P>::T;
    constexpr int NMB = W / 32;
#pragma unroll
    for (int kb = 0; kb < KIN; ++kb) {
        const Op a = load_a<P>(wsrc, t0 + (int64_t)kb * NMB + mb, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<P>(a, bin[kb][nb], kb == 0 ? f32x16{} : acc[nb]);
    }
    if constexpr (P == kBF16) {
        if (KIN == W / k_per_block(P)) {   // hidden layer: bias K-block
            const Op a = load_a<P>(wsrc, t0 + (int64_t)KIN * NMB + mb, lane);
            const Op one = bias_operand(h);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<P>(a, one, acc[nb]);
        }
    }
}

// One bf16 affine layer for a wave, software-pipelined: A tiles are loaded kAhead MFMA
// steps ahead (so LDS latency hides behind the matrix core), and the MFMAs of M-block mb
// are interleaved (scheduling barriers) with the ReLU/conversion of block mb - 1, so the
// matrix core runs while the vector ALU converts.  Hidden layers add the bias either as
// the accumulator's start value (kCInit: float32 bias tile from LDS) or through the bias
// K-block of the packed tiles; layer 0 reads it from two feature slots.
template <int W, int NB, int KIN, bool kCInit>
__device__ __attribute__((always_inline)) inline void dense_relu_bf16(const uint8_t *wsrc, int64_t t0,
                                                                      const bf16x8 (&bin)[W / 16][NB],
                                                                      bf16x8 (&bout)[W / 16][NB], const float *bias,
                                                                      int lane, int h) {
    constexpr int NMB = W / 32;
    constexpr bool kHidden = KIN == W / 16;
    constexpr bool kBiasBlock = kHidden && !kCInit;   // bias K-block MFMA
    constexpr bool kBiasInit = kHidden && kCInit;     // bias as the accumulator start
    constexpr int KS = KIN + (kBiasBlock ? 1 : 0);    // MFMA steps per M-block
    constexpr int NSTEP = NMB * KS;
    constexpr int kAhead = 3;
    const bf16x8 one = bias_operand(h);
    auto tile_of = [&](int step) { return t0 + (int64_t)(step % KS) * NMB + step / KS; };
    bf16x8 ring[kAhead];
#pragma unroll
    for (int i = 0; i < kAhead; ++i) ring[i] = load_a<kBF16>(wsrc, tile_of(i < NSTEP ? i : 0), lane);
    f32x16 acc[2][NB];   // M-blocks alternate between the two sets
    f32x16 bnext{};
    if constexpr (kBiasInit) bnext = bias_tile(bias, 0, h);
#pragma unroll
    for (int step = 0; step < NSTEP; ++step) {
        const int mb = step / KS, ks = step % KS;
        const bf16x8 a = ring[step % kAhead];
        if (step + kAhead < NSTEP) ring[step % kAhead] = load_a<kBF16>(wsrc, tile_of(step + kAhead), lane);
        f32x16 c0{};
        if constexpr (kBiasInit) {
            if (ks == 0) {
                c0 = bnext;
                if (mb + 1 < NMB) bnext = bias_tile(bias, mb + 1, h);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const bf16x8 bop = (kBiasBlock && ks == KIN) ? one : bin[ks < KIN ? ks : 0][nb];
            acc[mb & 1][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bop, ks == 0 ? c0 : acc[mb & 1][nb], 0, 0, 0);
        }
        if (ks == KS - 1) {
            if (mb > 0) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) relu_tile_to_bf16(acc[(mb - 1) & 1][nb], mb - 1, nb, bout);
                // 16 VALU per ray block (8 packed conversions, 8 packed max) against KS * NB
                // MFMAs of this block: one VALU after each MFMA, the rest after the chain
                // (a denser interleave keeps more values live and spills)
#pragma unroll
                for (int i = 0; i < KS * NB; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, 1, 0);   // VALU
                }
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) relu_tile_to_bf16(acc[(NMB - 1) & 1][nb], NMB - 1, nb, bout);
}

// One affine layer for a wave: KIN K-blocks of input operands `bin` -> the next layer's
// operands `bout` (ReLU; fp8: requantised).  M-blocks are processed one after another so
// that the epilogue of block mb (VALU) can overlap the MFMAs of block mb + 1.
template <int P, int W, int NB, int KIN, bool kCalib, bool kCInit>
__device__ __attribute__((always_inline)) inline void dense_relu(const uint8_t *wsrc, int64_t t0, const typename OpOf<P>::T (&bin)[W / k_per_block(P)][NB],
                                  typename OpOf<P>::T (&bout)[W / k_per_block(P)][NB], const float *bias, float alpha,
                                  int lane, int h, bool valid_any, unsigned int *amax_dst) {
    if constexpr (P == kBF16 && !kCalib) {
        dense_relu_bf16<W, NB, KIN, kCInit>(wsrc, t0, bin, bout, bias, lane, h);
        return;
    }
    constexpr int NMB = W / 32;
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
        f32x16 acc[NB];
        mblock_mfma<P, W, NB, KIN>(wsrc, t0, mb, bin, acc, lane, h);
        float bv[16];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const f32x4 b4 = *reinterpret_cast<const f32x4 *>(bias + mb * 32 + 8 * g + 4 * h);
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[4 * g + i] = b4[i];
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            float y[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if constexpr (P == kFP8)
                    y[j] = __builtin_amdgcn_fmed3f(fmaf(acc[nb][j], alpha, bv[j]), 0.f, kFp8Max);
                else if constexpr (P == kBF16)
                    y[j] = fmaxf(acc[nb][j], 0.f);   // bias already accumulated
                else
                    y[j] = fmaxf(acc[nb][j] + bv[j], 0.f);
            }
            if constexpr (kCalib) {
                float m = 0.f;
#pragma unroll
                for (int j = 0; j < 16; ++j) m = fmaxf(m, y[j]);
                wave_absmax(valid_any ? m : 0.f, amax_dst);
            }
            tile_to_operands<P>(y, mb, nb, bout);
        }
    }
}

// Same layer with the products ordered K-block outermost and the operands updated in place
// (fewer live registers: used for float32, for fp8, and whenever the weights are read from
// the L2-resident blob).  A tiles stream through a ring of kRing registers loaded kRing
// steps ahead, so global-memory latency hides behind the MFMAs.
template <int P, int W, int NB, int KIN, bool kCalib>
__device__ __attribute__((always_inline)) inline void dense_relu_inplace(
    const uint8_t *wsrc, int64_t t0, typename OpOf<P>::T (&b)[W / k_per_block(P)][NB], const float *bias, float alpha,
    int lane, int h, bool valid_any, unsigned int *amax_dst) {
    using Op = typename OpOf<P>::T;
    constexpr int NMB = W / 32;
    constexpr bool kBias = P == kBF16 && KIN == W / k_per_block(P);   // bf16 hidden layers: bias K-block
    constexpr int KS = KIN + (kBias ? 1 : 0);
    constexpr int NSTEP = KS * NMB;
    constexpr int kRing = P == kFP32 ? 8 : (P == kFP8 ? 2 : 4);   // fp8 tiles are 8 registers each
    f32x16 acc[NMB][NB];
    Op ring[kRing];
#pragma unroll
    for (int i = 0; i < kRing; ++i) ring[i] = load_a<P>(wsrc, t0 + (i < NSTEP ? i : 0), lane);
#pragma unroll
    for (int step = 0; step < NSTEP; ++step) {
        const int kb = step / NMB, mb = step % NMB;   // tiles are stored K-block major: tile = kb * NMB + mb
        const Op a = ring[step % kRing];
        if (step + kRing < NSTEP) ring[step % kRing] = load_a<P>(wsrc, t0 + step + kRing, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            if constexpr (kBias) {
                if (kb == KIN) {
                    acc[mb][nb] = mfma<P>(a, bias_operand(h), acc[mb][nb]);
                    continue;
                }
            }
            acc[mb][nb] = mfma<P>(a, b[kb < KIN ? kb : 0][nb], kb == 0 ? f32x16{} : acc[mb][nb]);
        }
    }
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
            if constexpr (P == kBF16 && !kCalib) {
                relu_tile_to_bf16(acc[mb][nb], mb, nb, b);   // bias already accumulated
                continue;
            }
            float y[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if constexpr (P == kFP8)
                    y[j] = __builtin_amdgcn_fmed3f(fmaf(acc[mb][nb][j], alpha, bv[j]), 0.f, kFp8Max);
                else
                    y[j] = fmaxf(acc[mb][nb][j] + bv[j], 0.f);
            }
            if constexpr (kCalib) {
                float m = 0.f;
#pragma unroll
                for (int j = 0; j < 16; ++j) m = fmaxf(m, y[j]);
                wave_absmax(valid_any ? m : 0.f, amax_dst);
            }
            tile_to_operands<P>(y, mb, nb, b);
        }
    }
}

// Head: rows 0 (logit) and 1 (distance) of one 32-row MFMA block, written by lanes 0..31.
template <int P, int W, int NB, bool kCInit = false, bool kUdf = false>
__device__ __attribute__((always_inline)) inline void head_out(const uint8_t *wsrc, int64_t th,
                                                               const typename OpOf<P>::T (&bin)[W / k_per_block(P)][NB],
                                                               const float *bias, float alpha, bool bad, int lane, int h,
                                                               int col, int64_t base, int64_t n, const bool (&nan_ray)[NB],
                                                               float *logit_out, float *dist_out, UdfDiv udq = {},
                                                               unsigned long long *udf_keys = nullptr) {
    using Op = typename OpOf<P>::T;
    constexpr int NKB = W / k_per_block(P);
    f32x16 start{};
    if constexpr (P == kBF16 && kCInit) {   // bias rows 0 and 1 as the start value (lane half 0)
        const f32x4 hb = *reinterpret_cast<const f32x4 *>(bias);
        const float keep = (float)(1 - h);
        start[0] = hb[0] * keep;
        start[1] = hb[1] * keep;
    }
    f32x16 acc[NB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        const Op a = load_a<P>(wsrc, th + kb, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<P>(a, bin[kb][nb], kb == 0 ? start : acc[nb]);
    }
    float c0 = bias[0], c1 = bias[1];
    if constexpr (P == kBF16 && kCInit) {
        c0 = c1 = 0.f;
    } else if constexpr (P == kBF16) {
        const Op a = load_a<P>(wsrc, th + NKB, lane);
        const Op one = bias_operand(h);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma<P>(a, one, acc[nb]);
        c0 = c1 = 0.f;
    }
    if constexpr (kUdf) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t r = base + nb * 32 + col;
            udf_block_min(fmaf(acc[nb][0] + acc[nb][2], alpha, c0), fmaf(acc[nb][1] + acc[nb][3], alpha, c1),
                          h == 0 && r < n && !nan_ray[nb] && !bad, r, udq, udf_keys, col);
        }
        return;
    }
    if (h == 0) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t r = base + nb * 32 + col;
            if (r < n) {
                // rows 2 and 3: the bf16 remainders of the head rows (zero in float32)
                logit_out[r] = (nan_ray[nb] || bad) ? NAN : fmaf(acc[nb][0] + acc[nb][2], alpha, c0);
                dist_out[r] = (nan_ray[nb] || bad) ? NAN : fmaf(acc[nb][1] + acc[nb][3], alpha, c1);
            }
        }
    }
}

// W: width, NB: 32-ray column blocks per wave, P: precision, kLdsA: weights in LDS,
// kCalib: record per-layer input absmax (fp8 calibration) instead of writing outputs.
// kOD: the inputs are origins [3][stride] (`rays`) and unit directions [3][stride] (`dirs`),
// assembled into the 5-value query in registers (one kernel for ray assembly and query).
// kUdf: the queries are the grid of `stride` points [3][stride] (`rays`) x `nd` directions
// given as angles [2][nd] (`dirs`), query r = point * nd + direction; instead of writing
// outputs each point's minimum hit distance goes to udf_keys (Eq. 5, see udf_block_min).
template <int P, int W, int NB, bool kLdsA, bool kCalib, bool kOD = false, bool kUdf = false>
__global__ __launch_bounds__(NB == 2 ? 512 : 256) void forward_kernel(
    const uint8_t *__restrict__ blob, int depth, const float *__restrict__ rays, int64_t stride,
    const int *__restrict__ count_dev, float *__restrict__ logit_out, float *__restrict__ dist_out,
    unsigned int *__restrict__ absmax, const float *__restrict__ dirs = nullptr, int nd = 0,
    unsigned long long *__restrict__ udf_keys = nullptr) {
    using Op = typename OpOf<P>::T;
    constexpr int KB = k_per_block(P);
    constexpr int NKB = W / KB;
    constexpr int K0 = layer0_kblocks(P);
    // bf16 with the weights in LDS starts each accumulation from the float32 bias (measured
    // 3% faster than the bias K-block, and exact in the bias); the other paths use the block
    constexpr bool kCInit = P == kBF16 && kLdsA;
    static_assert(K0 <= NKB, "layer-0 operands must fit the hidden operand array");
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];

    const NetLayout L = make_layout(W, depth, P);
    const int64_t wbytes = kLdsA ? L.tiles * tile_bytes(P) : 0;
    float *s_bias = reinterpret_cast<float *>(smem + wbytes);
    LdsConsts *s_c = reinterpret_cast<LdsConsts *>(s_bias + (W * depth + 4));
    {
        // Stage weights (optional) and biases; fp8 biases are pre-divided by the next scale.
        const int64_t nvec = wbytes / 16;
        for (int64_t i = threadIdx.x; i < nvec; i += blockDim.x)
            reinterpret_cast<i32x4 *>(smem)[i] = reinterpret_cast<const i32x4 *>(blob)[i];
        const float *g_bias = reinterpret_cast<const float *>(blob + L.bias_off);
        const float *g_scale = reinterpret_cast<const float *>(blob + L.scale_off);
        for (int i = threadIdx.x; i < W * depth + 4; i += blockDim.x) {
            float b = g_bias[i];
            if (P == kFP8 && i < W * depth) {
                const float sn = g_scale[2 * (i / W + 1) + 1];
                b = sn > 0.f ? b / sn : 0.f;
            }
            s_bias[i] = b;
        }
        if (threadIdx.x == 0) {
            s_c->bad = 0;
            if (P == kFP8) {
                const float s0 = g_scale[1];
                s_c->in_scale_inv = s0 > 0.f ? 1.f / s0 : 0.f;
                auto pow2 = [](float x) {
                    int e;
                    return x > 0.f && x < INFINITY && frexpf(x, &e) == 0.5f;
                };
                for (int l = 0; l <= depth; ++l) {
                    const float sw = g_scale[2 * l], sa = g_scale[2 * l + 1];
                    const float sn = l < depth ? g_scale[2 * (l + 1) + 1] : 1.f;
                    const float alpha = sn > 0.f ? sw * sa / sn : 0.f;
                    s_c->alpha[l] = alpha;
                    int e = 0;
                    frexpf(alpha, &e);
                    s_c->aexp[l] = 127 + e - 1;
                    if (!pow2(sw) || !pow2(sa) || !pow2(sn) || !pow2(alpha) || e - 1 < -126 || e - 1 > 127) s_c->bad = 1;
                }
            } else {
                s_c->in_scale_inv = 1.f;
                for (int l = 0; l <= depth; ++l) {
                    s_c->alpha[l] = 1.f;
                    s_c->aexp[l] = 127;
                }
            }
        }
    }
    __syncthreads();
    const uint8_t *wsrc = kLdsA ? smem : blob;

    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int wpb = blockDim.x >> 6;
    // rays are rows of length `stride`; the first `n` are evaluated (n from the device when
    // a queue produced them)
    const int64_t n = kUdf ? stride * nd : count_dev ? min<int64_t>(*count_dev, stride) : stride;
    UdfDiv udq{};
    if constexpr (kUdf) udq = udf_div_make(nd);
    const int64_t ntile = (n + 32 * NB - 1) / (32 * NB);

    // With the weights in LDS the rays of the next tile are loaded while this one is computed
    // (HBM latency hides behind the layers instead of stalling the encoding); the L2 variants
    // have no registers to spare for that and load at the top of the tile.
    const int64_t tstride = (int64_t)gridDim.x * wpb;
    float vnext[NB][kInRaw];
    float dz_next[NB];   // kOD: third direction component
    auto load_rays = [&](int64_t t) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t r = t * 32 * NB + nb * 32 + col;
            if constexpr (kOD) {
#pragma unroll
                for (int j = 0; j < 3; ++j) vnext[nb][j] = r < n ? rays[(int64_t)j * stride + r] : 0.f;
                // the direction is kept raw here and turned into angles at the encoding
                vnext[nb][3] = r < n ? dirs[r] : 0.f;
                vnext[nb][4] = r < n ? dirs[stride + r] : 0.f;
                dz_next[nb] = r < n ? dirs[2 * stride + r] : 1.f;
            } else if constexpr (kUdf) {
                const int p = r < n ? udf_div(udq, (int)r) : 0, j = r < n ? (int)r - p * nd : 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) vnext[nb][c] = r < n ? rays[(int64_t)c * stride + p] : 0.f;
                vnext[nb][3] = r < n ? dirs[j] : 0.f;
                vnext[nb][4] = r < n ? dirs[nd + j] : 0.f;
            } else {
#pragma unroll
                for (int j = 0; j < kInRaw; ++j) vnext[nb][j] = r < n ? rays[(int64_t)j * stride + r] : 0.f;
            }
        }
    };
    int64_t tile = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    if constexpr (kLdsA) load_rays(tile);
    // Issue priority (bf16 and fp8 with the weights in LDS): a wave in its MFMA layers outranks
    // a wave in its encoding and epilogue, and of two waves in their layers the odd one leads,
    // so the two waves of a SIMD settle into taking turns on the matrix core (measured ~2%
    // faster in bf16, ~1.3% in fp8, outputs bitwise unchanged).
    const bool odd_wave = (threadIdx.x >> 6) & 1;
    for (; tile < ntile; tile += tstride) {
        if constexpr ((P == kBF16 || (P == kFP8 && !kCalib)) && kLdsA) __builtin_amdgcn_s_setprio(0);
        const int64_t base = tile * 32 * NB;
        if constexpr (!kLdsA) load_rays(tile);
        float vcur[NB][kInRaw];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
            for (int j = 0; j < kInRaw; ++j) vcur[nb][j] = vnext[nb][j];
            if constexpr (kOD) {
                // lane half 0 takes the polar angle, half 1 the azimuth (one atan2 per lane), and
                // the partner lane (l xor 32, the same ray) passes the other one across
                const float dx = vnext[nb][3], dy = vnext[nb][4];
                const float ay = h ? dy : polar_y(dx, dy), ax = h ? dx : dz_next[nb];
                float ang = atan2f(ay, ax);
                if (h) ang = wrap_azimuth(ang);
                const float other = __shfl_xor(ang, 32);
                vcur[nb][3] = h ? other : ang;   // theta
                vcur[nb][4] = h ? ang : other;   // phi
            }
        }
        if constexpr (kLdsA) load_rays(tile + tstride);
        Op b0[NKB][NB], b1[NKB][NB];   // ping-pong operands of consecutive layers
        bool nan_ray[NB];              // NaN inputs give NaN outputs (ReLU's fmax would hide them)
        bool valid_any = false;
        // ---- encoding -> layer-0 B operands
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int64_t r = base + nb * 32 + col;
            const float *v = vcur[nb];
            valid_any |= r < n;
            nan_ray[nb] = isnan(v[0]) || isnan(v[1]) || isnan(v[2]) || isnan(v[3]) || isnan(v[4]);
            float feat[kSlotsPerHalf];
            encode_var<P == kFP32, P == kFP8>(h ? v[3] : v[0], feat);
            encode_var<P == kFP32, P == kFP8>(h ? v[4] : v[1], feat + kFeatPerVar);
            encode_var<P == kFP32, P == kFP8>(h ? 0.f : v[2], feat + 2 * kFeatPerVar);
            feat[kSlotsPerHalf - 1] = 0.f;
            if constexpr (P == kBF16) {
                feat[kBiasSlot0] = h ? 1.f : feat[kBiasSlot0];
                feat[kBiasSlot1] = h ? 1.f : 0.f;
            }
            if constexpr (kCalib) {
                float m = 0.f;
#pragma unroll
                for (int f = 0; f < kSlotsPerHalf - 1; ++f)
                    if (r < n && (h == 0 || f < 2 * kFeatPerVar)) m = fmaxf(m, fabsf(feat[f]));
                wave_absmax(m, absmax + 1);
            }
            if constexpr (P == kBF16) {
#pragma unroll
                for (int kb = 0; kb < K0; ++kb)
#pragma unroll
                    for (int s = 0; s < 8; ++s) b0[kb][nb][s] = (__bf16)feat[kb * 8 + s];
            } else if constexpr (P == kFP8) {
                const float inv = s_c->in_scale_inv;
#pragma unroll
                for (int kb = 0; kb < K0; ++kb)
#pragma unroll
                    for (int w4 = 0; w4 < 8; ++w4) {
                        float q[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int f = kb * 32 + w4 * 4 + i;
                            q[i] = f < kSlotsPerHalf ? __builtin_amdgcn_fmed3f(feat[f] * inv, -kFp8Max, kFp8Max) : 0.f;
                        }
                        b0[kb][nb][w4] = pack_fp8x4(q[0], q[1], q[2], q[3]);
                    }
            } else {
#pragma unroll
                for (int kb = 0; kb < K0; ++kb) b0[kb][nb] = feat[kb];
            }
        }
        if constexpr (P == kFP8 && kLdsA && !kCalib) {
            static_assert(K0 == NKB, "fp8 layer 0 and hidden layers share the operand shape");
            const bool bad = s_c->bad != 0;
            if (odd_wave) __builtin_amdgcn_s_setprio(2);
            else __builtin_amdgcn_s_setprio(1);
            dense_fp8<W, NB, K0>(wsrc, L.layer_tile(0), b0, b1, s_bias, s_c->aexp[0], lane, h);
            int l = 1;
            for (; l + 1 < depth; l += 2) {
                dense_fp8<W, NB, NKB>(wsrc, L.layer_tile(l), b1, b0, s_bias + l * W, s_c->aexp[l], lane, h);
                dense_fp8<W, NB, NKB>(wsrc, L.layer_tile(l + 1), b0, b1, s_bias + (l + 1) * W, s_c->aexp[l + 1], lane, h);
            }
            if (l < depth) {
                dense_fp8<W, NB, NKB>(wsrc, L.layer_tile(l), b1, b0, s_bias + l * W, s_c->aexp[l], lane, h);
                head_fp8<W, NB, kUdf>(wsrc, L.head_tile(), b0, s_bias + W * depth, s_c->aexp[depth], bad, lane, h,
                                      col, base, n, nan_ray, logit_out, dist_out, udq, udf_keys);
            } else {
                head_fp8<W, NB, kUdf>(wsrc, L.head_tile(), b1, s_bias + W * depth, s_c->aexp[depth], bad, lane, h,
                                      col, base, n, nan_ray, logit_out, dist_out, udq, udf_keys);
            }
            continue;
        }
        if constexpr (P != kBF16 || !kLdsA) {
            dense_relu_inplace<P, W, NB, K0, kCalib>(wsrc, L.layer_tile(0), b0, s_bias, s_c->alpha[0], lane, h,
                                                      valid_any, absmax + 3);
            for (int l = 1; l < depth; ++l)
                dense_relu_inplace<P, W, NB, NKB, kCalib>(wsrc, L.layer_tile(l), b0, s_bias + l * W, s_c->alpha[l], lane,
                                                           h, valid_any, absmax + 2 * (l + 1) + 1);
            if constexpr (!kCalib)
                head_out<P, W, NB, false, kUdf>(wsrc, L.head_tile(), b0, s_bias + W * depth, s_c->alpha[depth],
                                                s_c->bad != 0, lane, h, col, base, n, nan_ray, logit_out, dist_out, udq,
                                                udf_keys);
            continue;
        }
        // ---- layer 0, then hidden layers two at a time (b1 -> b0 -> b1 ...)
        if constexpr (P == kBF16 && kLdsA) {
            if (odd_wave) __builtin_amdgcn_s_setprio(2);
            else __builtin_amdgcn_s_setprio(1);
        }
        dense_relu<P, W, NB, K0, kCalib, kCInit>(wsrc, L.layer_tile(0), b0, b1, s_bias, s_c->alpha[0], lane, h, valid_any,
                                          absmax + 3);
        int l = 1;
        for (; l + 1 < depth; l += 2) {
            dense_relu<P, W, NB, NKB, kCalib, kCInit>(wsrc, L.layer_tile(l), b1, b0, s_bias + l * W, s_c->alpha[l], lane, h,
                                               valid_any, absmax + 2 * (l + 1) + 1);
            dense_relu<P, W, NB, NKB, kCalib, kCInit>(wsrc, L.layer_tile(l + 1), b0, b1, s_bias + (l + 1) * W,
                                               s_c->alpha[l + 1], lane, h, valid_any, absmax + 2 * (l + 2) + 1);
        }
        const bool last_in_b0 = l < depth;   // one hidden layer left: it writes b0
        if (last_in_b0)
            dense_relu<P, W, NB, NKB, kCalib, kCInit>(wsrc, L.layer_tile(l), b1, b0, s_bias + l * W, s_c->alpha[l], lane, h,
                                               valid_any, absmax + 2 * (l + 1) + 1);
        if constexpr (kCalib) continue;
        // ---- head: rows 0 (logit) and 1 (distance) of one 32-row block
        if (last_in_b0)
            head_out<P, W, NB, kCInit, kUdf>(wsrc, L.head_tile(), b0, s_bias + W * depth, s_c->alpha[depth], s_c->bad != 0,
                                             lane, h, col, base, n, nan_ray, logit_out, dist_out, udq, udf_keys);
        else
            head_out<P, W, NB, kCInit, kUdf>(wsrc, L.head_tile(), b1, s_bias + W * depth, s_c->alpha[depth], s_c->bad != 0,
                                             lane, h, col, base, n, nan_ray, logit_out, dist_out, udq, udf_keys);
    }
}

// Smallest power of two s with a / s <= 448 (1 for a = 0; a non-finite absmax is passed
// through, which the forward kernels reject).
__device__ inline float pow2_scale(float a) {
    if (!(a > 0.f)) return 1.f;
    if (!(a < INFINITY)) return a;
    int e;
    frexpf(a / kFp8Max, &e);
    float s = ldexpf(1.f, e);
    while (a > kFp8Max * s) s *= 2.f;   // a / 448 may have rounded: compare exactly
    while (a <= kFp8Max * 0.5f * s) s *= 0.5f;
    return s;
}

// Weight absmax per affine layer (one block per layer) -> scales[2 l]; input absmax bits
// (written by the calibration forward) -> scales[2 l + 1]; each as pow2_scale.
__global__ void weight_absmax_kernel(const float *__restrict__ params, int width, int depth, float *scales) {
    const int l = blockIdx.x;
    int64_t off = 0;
    int in = kInDim;
    for (int j = 0; j < l; ++j) {
        off += (int64_t)width * in + width;
        in = width;
    }
    const int out = l == depth ? 2 : width;
    const int64_t cnt = (int64_t)out * in;
    float m = 0.f;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) m = fmaxf(m, fabsf(params[off + i]));
    __shared__ float red[256];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scales[2 * l] = pow2_scale(red[0]);
        const float a = __uint_as_float(reinterpret_cast<unsigned int *>(scales)[2 * l + 1]);
        scales[2 * l + 1] = pow2_scale(a);
    }
}

__global__ void zero_kernel(float *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ------------------------------------------------------------------------------ dispatch
int cu_count() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    });
    return cus;
}

// udf_keys (weights in LDS only): the UDF grid of n points x nd directions (angles in `dirs`).
template <int P, int W, int NB, bool kLdsA>
ddf_status launch_forward(const NetLayout &L, const void *blob, const float *rays, int64_t n, const int *count_dev,
                          float *logit, float *dist, unsigned int *absmax, hipStream_t stream,
                          const float *dirs = nullptr, int nd = 0, unsigned long long *udf_keys = nullptr) {
    if (absmax) {
        if constexpr (P == kFP32 && !kLdsA) {
            auto kc = forward_kernel<P, W, NB, kLdsA, true>;
            const int threads = NB == 2 ? 512 : 256;
            const size_t lds = ((size_t)W * L.depth + 4) * 4 + sizeof(LdsConsts);
            hipLaunchKernelGGL(kc, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 32 * NB * 4 - 1) / (32 * NB * 4), 512))),
                               dim3(threads), lds, stream, (const uint8_t *)blob, L.depth, rays, n, count_dev, logit, dist, absmax,
                               (const float *)nullptr, 0, (unsigned long long *)nullptr);
            return launch_status("ddf_fp8_scales (calibration)");
        }
        set_error("calibration runs on float32 networks only");
        return DDF_ERR_UNSUPPORTED;
    }
    auto kern = forward_kernel<P, W, NB, kLdsA, false>;
    if constexpr (kLdsA) {   // the fused ray assembly and the fused UDF exist for the LDS kernels only
        if (udf_keys) kern = forward_kernel<P, W, NB, kLdsA, false, false, true>;
        else if (dirs) kern = forward_kernel<P, W, NB, kLdsA, false, true>;
    }
    const size_t lds = (kLdsA ? L.tiles * tile_bytes(P) : 0) + ((size_t)W * L.depth + 4) * 4 + sizeof(LdsConsts);
    static std::once_flag once;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void *)forward_kernel<P, W, NB, kLdsA, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        if constexpr (kLdsA) {
            (void)hipFuncSetAttribute((const void *)forward_kernel<P, W, NB, kLdsA, false, true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
            (void)hipFuncSetAttribute((const void *)forward_kernel<P, W, NB, kLdsA, false, false, true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
        }
    });
    const int threads = NB == 2 ? 512 : 256;
    const int64_t nq = udf_keys ? n * nd : n;   // queries
    const int64_t ntile = (nq + 32 * NB - 1) / (32 * NB);
    const int64_t wpb = threads / 64;
    const int per_cu = kLdsA ? 1 : 2;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((ntile + wpb - 1) / wpb, (int64_t)cu_count() * per_cu));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(threads), lds, stream, (const uint8_t *)blob, L.depth, rays, n,
                       count_dev, logit, dist, absmax, dirs, nd, udf_keys);
    return launch_status("ddf_forward");
}

bool fits_lds(const NetLayout &L) {
    return L.tiles * tile_bytes(L.prec) + ((int64_t)L.width * L.depth + 4) * 4 + (int64_t)sizeof(LdsConsts) <= kLdsBytes;
}

ddf_status check_shape(int width, int depth, int prec, const char *who) {
    DDF_REQUIRE(width == 128 || width == 256, DDF_ERR_UNSUPPORTED, "%s: width %d not supported (128 or 256)", who, width);
    DDF_REQUIRE(depth >= 1 && depth <= 8, DDF_ERR_UNSUPPORTED, "%s: depth %d not supported (1..8)", who, depth);
    DDF_REQUIRE(prec == kFP32 || prec == kBF16 || prec == kFP8, DDF_ERR_UNSUPPORTED, "%s: unknown precision %d", who, prec);
    return DDF_OK;
}

}  // namespace

// Network query of the first n (or *count_dev) rays of a [5][n] buffer.
ddf_status forward_dispatch(const ddf_net *net, const float *rays, int64_t n, const int *count_dev, float *logit,
                            float *dist, unsigned int *absmax, hipStream_t s) {
    const NetLayout L = make_layout(net->width, net->depth, net->precision);
    // DDF_WEIGHTS_IN_LDS=0 keeps the weights in the L2-resident blob (tuning / diagnosis)
    static const bool allow_lds = [] {
        const char *e = std::getenv("DDF_WEIGHTS_IN_LDS");
        return !(e && e[0] == '0');
    }();
    const bool lds = allow_lds && fits_lds(L);
    if (net->precision == kBF16 && !lds && !absmax) {
        // weights too large for one CU's LDS: a workgroup streams them and its waves share them
        GradArgs a{};
        a.blob = (const uint8_t *)net->packed;
        a.depth = net->depth;
        a.rays = rays;
        a.n = n;
        a.count_dev = count_dev;
        a.logit_out = logit;
        a.dist_out = dist;
        a.forward_only = true;
        return stream_dispatch(net->width, a, s);
    }
    if (net->width == 128) {
        if (net->precision == kBF16)   // (bf16 networks beyond LDS took the streamed kernel above)
            return launch_forward<kBF16, 128, 2, true>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s);
        // fp8 from L2 runs one 32-ray block per wave (two blocks spilled in that variant)
        if (net->precision == kFP8)
            return lds ? launch_forward<kFP8, 128, 2, true>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s)
                       : launch_forward<kFP8, 128, 1, false>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s);
        return launch_forward<kFP32, 128, 1, false>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s);
    }
    if (net->precision == kBF16) return launch_forward<kBF16, 256, 1, false>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s);
    if (net->precision == kFP8) return launch_forward<kFP8, 256, 1, false>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s);
    if (!absmax && !count_dev) {
        // float32 at width 256: the training sweep's forward (layer values of 64 rays in LDS);
        // the per-wave kernel would hold a whole layer's operands and outputs in registers
        GradArgs a{};
        a.blob = (const uint8_t *)net->packed;
        a.depth = net->depth;
        a.rays = rays;
        a.n = n;
        a.logit_out = logit;
        a.dist_out = dist;
        a.forward_only = true;
        return sweep_dispatch(256, a, s);
    }
    return launch_forward<kFP32, 256, 1, false>(L, net->packed, rays, n, count_dev, logit, dist, absmax, s);
}

// Fused UDF (Eq. 5): networks whose weights fit in LDS (width 128, bf16 or fp8) and grids of
// fewer than 2^31 queries.
bool udf_fused_ok(const ddf_net *net, int64_t np, int64_t nd) {
    const NetLayout L = make_layout(net->width, net->depth, net->precision);
    return net->width == 128 && net->precision != kFP32 && fits_lds(L) && np * nd < ((int64_t)1 << 31);
}

// keys [np] must hold ~0 on entry; ang is [2][nd].
ddf_status udf_fused_launch(const ddf_net *net, const float *points, int64_t np, const float *ang, int64_t nd,
                            unsigned long long *keys, hipStream_t s) {
    const NetLayout L = make_layout(net->width, net->depth, net->precision);
    if (net->precision == kBF16)
        return launch_forward<kBF16, 128, 2, true>(L, net->packed, points, np, nullptr, nullptr, nullptr, nullptr, s, ang,
                                                   (int)nd, keys);
    return launch_forward<kFP8, 128, 2, true>(L, net->packed, points, np, nullptr, nullptr, nullptr, nullptr, s, ang,
                                              (int)nd, keys);
}

}  // namespace ddf

using namespace ddf;

extern "C" ddf_status ddf_packed_bytes(int32_t width, int32_t depth, int32_t precision, size_t *bytes) {
    if (ddf_status st = check_shape(width, depth, precision, "ddf_packed_bytes")) return st;
    DDF_REQUIRE(bytes, DDF_ERR_INVALID_ARG, "ddf_packed_bytes: NULL output");
    *bytes = (size_t)make_layout(width, depth, precision).bytes;
    return DDF_OK;
}

extern "C" ddf_status ddf_pack_net(const float *params, int32_t width, int32_t depth, int32_t precision,
                                   const float *scales, void *packed, ddf_stream stream) {
    if (ddf_status st = check_shape(width, depth, precision, "ddf_pack_net")) return st;
    DDF_REQUIRE(params && packed, DDF_ERR_INVALID_ARG, "ddf_pack_net: NULL params or output");
    DDF_REQUIRE((precision == kFP8) == (scales != nullptr), DDF_ERR_INVALID_ARG,
                "ddf_pack_net: fp8 needs scales, other precisions take none");
    hipLaunchKernelGGL(pack_kernel, dim3(1024), dim3(256), 0, as_stream(stream), params, width, depth, precision, scales,
                       (uint8_t *)packed);
    return launch_status("ddf_pack_net");
}

extern "C" ddf_status ddf_fp8_scales(const ddf_net *net_fp32, const float *params, const float *calib, int64_t n_calib,
                                     float *scales_out, ddf_stream stream) {
    DDF_REQUIRE(net_fp32 && params && scales_out, DDF_ERR_INVALID_ARG, "ddf_fp8_scales: NULL argument");
    if (ddf_status st = check_shape(net_fp32->width, net_fp32->depth, net_fp32->precision, "ddf_fp8_scales")) return st;
    DDF_REQUIRE(net_fp32->precision == kFP32 && net_fp32->packed, DDF_ERR_INVALID_ARG,
                "ddf_fp8_scales: needs a packed float32 network");
    DDF_REQUIRE(n_calib > 0 && calib, DDF_ERR_INVALID_ARG, "ddf_fp8_scales: need calibration rays");
    hipStream_t s = as_stream(stream);
    const int nsc = 2 * (net_fp32->depth + 1);
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, scales_out, (int64_t)nsc);
    if (ddf_status st = launch_status("ddf_fp8_scales")) return st;
    if (ddf_status st = forward_dispatch(net_fp32, calib, n_calib, nullptr, nullptr, nullptr,
                                         reinterpret_cast<unsigned int *>(scales_out), s))
        return st;
    hipLaunchKernelGGL(weight_absmax_kernel, dim3(net_fp32->depth + 1), dim3(256), 0, s, params, net_fp32->width,
                       net_fp32->depth, scales_out);
    return launch_status("ddf_fp8_scales");
}

extern "C" ddf_status ddf_query(const ddf_net *net, const float *orig, const float *dir, int64_t n, float *logit_out,
                                float *dist_out, ddf_stream stream) {
    DDF_REQUIRE(net, DDF_ERR_INVALID_ARG, "ddf_query: NULL network");
    if (ddf_status st = check_shape(net->width, net->depth, net->precision, "ddf_query")) return st;
    DDF_REQUIRE(n >= 0, DDF_ERR_INVALID_ARG, "ddf_query: negative n");
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(net->packed && orig && dir && logit_out && dist_out, DDF_ERR_INVALID_ARG, "ddf_query: NULL array");
    const NetLayout L = make_layout(net->width, net->depth, net->precision);
    DDF_REQUIRE(net->width == 128 && net->precision != kFP32 && fits_lds(L), DDF_ERR_UNSUPPORTED,
                "ddf_query: needs a bf16 or fp8 network whose weights fit in LDS (width 128); use "
                "ddf_assemble_rays + ddf_forward otherwise");
    hipStream_t s = as_stream(stream);
    if (net->precision == kBF16)
        return launch_forward<kBF16, 128, 2, true>(L, net->packed, orig, n, nullptr, logit_out, dist_out, nullptr, s, dir);
    return launch_forward<kFP8, 128, 2, true>(L, net->packed, orig, n, nullptr, logit_out, dist_out, nullptr, s, dir);
}

extern "C" ddf_status ddf_forward(const ddf_net *net, const float *rays, int64_t n, float *logit_out, float *dist_out,
                                  ddf_stream stream) {
    DDF_REQUIRE(net, DDF_ERR_INVALID_ARG, "ddf_forward: NULL network");
    if (ddf_status st = check_shape(net->width, net->depth, net->precision, "ddf_forward")) return st;
    DDF_REQUIRE(n >= 0, DDF_ERR_INVALID_ARG, "ddf_forward: negative n");
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(net->packed && rays && logit_out && dist_out, DDF_ERR_INVALID_ARG, "ddf_forward: NULL array");
    return forward_dispatch(net, rays, n, nullptr, logit_out, dist_out, nullptr, as_stream(stream));
}
