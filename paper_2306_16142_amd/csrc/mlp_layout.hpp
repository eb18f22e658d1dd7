// Packed-network layout shared by the packing kernel and the forward kernels.
//
// The network (Sec. IV-A, MLP_w) has `depth` hidden ReLU layers of `width` units on the
// 65 Fourier features of a ray and a 2-unit head (hit logit, distance).  Its affine
// layers run on 32x32 MFMA tiles with the weight matrix as operand A (rows = output
// units) and a wave's rays as operand B (columns = rays), so that a layer's result,
// which leaves lane l holding column l % 32 and rows 8 g + 4 (l / 32) + i (g, i < 4) of
// every 32-row block, is already the B operand of the next layer once the contraction
// index k is renumbered to match.  The renumbering is folded into the packed weights:
// the blob stores, per (layer, K-block, M-block), the 64 lanes' A operands in exactly
// the order each lane reads them.
//
// Layer 0 reads the Fourier features.  Lanes of half h = l / 32 encode their own rays'
// variables: half 0 the three origin coordinates, half 1 the two angles (and one unused
// slot group); each variable gives 13 features (raw, sin 2^k v, cos 2^k v, k = 0..5),
// so every half holds 40 feature slots (39 used).
#pragma once
#include <cstddef>
#include <cstdint>

namespace ddf {

enum Precision { kFP32 = 0, kBF16 = 1, kFP8 = 2 };

constexpr int kInRaw = 5;
constexpr int kNFreq = 6;
constexpr int kInDim = 65;
constexpr int kFeatPerVar = 13;     // raw + 6 sin + 6 cos
constexpr int kSlotsPerHalf = 40;   // 3 variables x 13 features + 1 pad

// Contraction depth per MFMA and A-operand bytes per lane.
__host__ __device__ constexpr int k_per_block(int prec) { return prec == kBF16 ? 16 : prec == kFP8 ? 64 : 2; }
__host__ __device__ constexpr int slots_per_lane(int prec) { return prec == kBF16 ? 8 : prec == kFP8 ? 32 : 1; }
__host__ __device__ constexpr int tile_bytes(int prec) { return prec == kBF16 ? 1024 : prec == kFP8 ? 2048 : 256; }
__host__ __device__ constexpr int layer0_kblocks(int prec) { return prec == kBF16 ? 5 : prec == kFP8 ? 2 : 40; }
// bf16 adds each layer's bias inside the MFMA chain: hidden layers and the head get one extra
// K-block whose A tile holds the bias split as bf16 hi + lo in slots 0 and 1 of lane half 0
// (the matching B operand is the constant 1, 1 there); layer 0 uses two unused feature
// slots of lane half 1 (kBiasSlot0/1).  fp32 adds it in the epilogue, fp8 folds it into the
// requantising fma.
__host__ __device__ constexpr int bias_kblocks(int prec) { return prec == kBF16 ? 1 : 0; }
constexpr int kBiasSlot0 = 38;
constexpr int kBiasSlot1 = 39;

// Blob sections: forward A tiles | biases | fp8 scales | (fp32 / bf16 only) transposed
// A tiles of the input-gradient sweep | the head's two weight rows in float32.
constexpr int kGradRowBlocks0 = 3;   // layer-0 transposed product: 96 rows = 48 feature slots per half

struct NetLayout {
    int width, depth, prec;
    int nmb, nkb, k0;           // M-blocks, hidden K-blocks, layer-0 K-blocks
    int xkb;                    // extra bias K-blocks of hidden layers and the head
    int64_t tiles;              // forward A tiles in total
    int64_t bias_off;           // byte offset of float bias[width*depth + 4]
    int64_t scale_off;          // byte offset of float scales[2*(depth+1)] (fp8)
    int64_t grad_tiles;         // transposed A tiles (0 for fp8)
    int64_t grad_off;           // byte offset of the transposed tiles
    int64_t head_rows_off;      // byte offset of float head_rows[2][width]
    int64_t bytes;              // total blob size

    __host__ __device__ int64_t layer_tile(int l) const {
        return l == 0 ? 0 : (int64_t)k0 * nmb + (int64_t)(l - 1) * (nkb + xkb) * nmb;
    }
    __host__ __device__ int64_t head_tile() const { return layer_tile(depth); }
    // Transposed tiles: layer 0 (kGradRowBlocks0 x nkb), then layers 1..depth-1 (nmb x nkb each).
    __host__ __device__ int64_t grad_layer_tile(int l) const {
        return l == 0 ? 0 : (int64_t)kGradRowBlocks0 * nkb + (int64_t)(l - 1) * nkb * nmb;
    }
};

__host__ __device__ inline NetLayout make_layout(int width, int depth, int prec) {
    NetLayout L;
    L.width = width;
    L.depth = depth;
    L.prec = prec;
    L.nmb = width / 32;
    L.nkb = width / k_per_block(prec);
    L.k0 = layer0_kblocks(prec);
    L.xkb = bias_kblocks(prec);
    L.tiles = (int64_t)L.k0 * L.nmb + (int64_t)(depth - 1) * (L.nkb + L.xkb) * L.nmb + L.nkb + L.xkb;
    L.bias_off = L.tiles * tile_bytes(prec);
    L.scale_off = L.bias_off + ((int64_t)width * depth + 4) * 4;
    int64_t sbytes = (int64_t)2 * (depth + 1) * 4;
    L.grad_off = L.scale_off + ((sbytes + 15) / 16) * 16;
    L.grad_tiles = prec == kFP8 ? 0 : (int64_t)kGradRowBlocks0 * L.nkb + (int64_t)(depth - 1) * L.nkb * L.nmb;
    L.head_rows_off = L.grad_off + L.grad_tiles * tile_bytes(prec);
    L.bytes = L.head_rows_off + (prec == kFP8 ? 0 : (int64_t)2 * width * 4);
    return L;
}

// Column of the 65-feature input read by layer-0 feature slot f (0..39) of lane half h,
// or -1 for an unused slot.  Feature order of the input: 5 raw values, then sin(2^k v_j)
// for k = 0..5 (outer) and j = 0..4 (inner), then cos(2^k v_j) in the same order.
__host__ __device__ inline int feature_column(int h, int f) {
    if (f >= 3 * kFeatPerVar) return -1;
    const int var = f / kFeatPerVar, r = f % kFeatPerVar;
    const int j = h == 0 ? var : (var < 2 ? 3 + var : -1);
    if (j < 0) return -1;
    if (r == 0) return j;
    if (r <= kNFreq) return kInRaw + kInRaw * (r - 1) + j;
    return kInRaw + kInRaw * kNFreq + kInRaw * (r - 1 - kNFreq) + j;
}

// Layer-0 feature slot of (K-block kb, lane half h, operand slot s).
__host__ __device__ inline int layer0_feature(int prec, int kb, int s) {
    return kb * slots_per_lane(prec) + s;   // fp32: one slot per K-step
}

// Layer-0 feature slot (of the owning lane half) of row m of the transposed layer-0 product.
__host__ __device__ inline int grad_row_half(int m) { return (m % 8) / 4; }
__host__ __device__ inline int grad_row_feature(int m) { return (m / 32) * 16 + ((m % 32) / 8) * 4 + (m % 4); }

// Previous-layer unit fed by (K-block kb, lane half h, operand slot s) of a hidden or head layer.
__host__ __device__ inline int prev_unit(int prec, int kb, int h, int s) {
    if (prec == kBF16) return 32 * (kb / 2) + 16 * (kb % 2) + 8 * (s / 4) + 4 * h + (s % 4);
    if (prec == kFP8) return 32 * (2 * kb + s / 16) + 8 * ((s % 16) / 4) + 4 * h + (s % 4);
    const int j = kb % 16;   // fp32: K-step kb takes accumulator j of M-block kb / 16
    return 32 * (kb / 16) + 8 * (j / 4) + 4 * h + (j % 4);
}

}  // namespace ddf
