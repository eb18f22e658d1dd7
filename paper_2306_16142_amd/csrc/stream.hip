// Network query and input gradient (Sec. IV-A query, Eq. 3 normals) for bf16 networks whose
// packed weights do not fit in one CU's LDS: width 256, or width 128 deeper than four layers.
//
// A workgroup evaluates 256 rays at a time and streams the weight tiles through an LDS ring
// that all its waves read.  One "phase" is one 32-row M-block of one layer (its K-blocks,
// plus the bias K-block of a hidden layer).  At the start of phase p each wave issues its
// share of phase p + 2 as buffer loads that write LDS directly and waits for them
// before the next barrier, which publishes the stages: at width 128 one barrier per phase
// (three stages), at width 256 one per pair of phases (four stages).  The table lookup that locates a phase's tiles is done one phase
// early, across the previous barrier, so a phase begins with its loads and its MFMA chain.
// Every wave reads each weight tile from LDS, and the workgroup reads it from L2 once per
// 256 rays (the per-wave kernel read it once per 32 or 64).
//
// Per wave everything else is as in the other network kernels: the Fourier encoding in
// registers, layer outputs kept in the accumulators and converted into the next layer's B
// operands (ReLU on packed bf16), ReLU masks in LDS (16 bits per lane and tile) for the
// reverse sweep, the transposed tiles for the adjoints, and the chain rule through the
// features in registers.
#include <cmath>
#include <mutex>

#include "common.hpp"
#include "grad_args.hpp"
#include "mlp_device.hpp"
#include "mlp_layout.hpp"
#include "tuning.hpp"

namespace ddf {
namespace {

// Width 128: four waves of two 32-ray blocks, two workgroups per CU.  Width 256: eight waves
// of one block (two ray blocks would need about 380 registers per lane).
template <int W>
struct Geo {
    static constexpr int kWaves = W == 256 ? 8 : 4;
    static constexpr int kNB = W == 256 ? 1 : 2;
};
constexpr int kRaysPerTile = 256;
// Width 256 runs its phases in pairs between barriers with a four-stage ring; width 128 (whose
// two workgroups per CU need the smaller ring) one phase per barrier with three stages.
template <int W>
struct Ring {
    static constexpr bool kPair = W == 256;
    static constexpr int kStages = kPair ? 4 : 3;
};
constexpr int kMaxStreamLds = 160 * 1024;
constexpr int kMaxPhases = 8 * 8 + 1 + 7 * 8 + kGradRowBlocks0;   // width 256, depth 8, gradient

typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(1))) const uint8_t gbl_u8;

template <int W>
__host__ __device__ inline int phases_of(int depth, bool grad) {
    constexpr int NMB = W / 32;
    return NMB * depth + 1 + (grad ? (depth - 1) * NMB + kGradRowBlocks0 : 0);
}

// Phase q of a network's program -> (byte offset of its first tile in the blob, byte stride
// between its tiles, number of tiles).  Order: layer 0 (NMB phases of 5 K-blocks), hidden
// layers (NMB phases of NKB + 1 K-blocks, the last the bias block), the head (one phase of
// NKB + 1), then for gradients the transposed hidden layers from the top (NMB phases of NKB)
// and the transposed layer 0 (kGradRowBlocks0 phases of NKB).
template <int W>
__device__ inline void phase_entry(int depth, int q, int &off, int &stride, int &ks) {
    constexpr int NMB = W / 32, NKB = W / 16;
    const NetLayout L = make_layout(W, depth, kBF16);
    const int tb = tile_bytes(kBF16);
    if (q < NMB) {
        off = (int)((L.layer_tile(0) + q) * tb);
        ks = layer0_kblocks(kBF16);
        stride = NMB * tb;
        return;
    }
    q -= NMB;
    if (q < (depth - 1) * NMB) {
        off = (int)((L.layer_tile(1 + q / NMB) + q % NMB) * tb);
        ks = NKB + 1;
        stride = NMB * tb;
        return;
    }
    q -= (depth - 1) * NMB;
    if (q == 0) {
        off = (int)(L.head_tile() * tb);
        ks = NKB + 1;
        stride = tb;
        return;
    }
    q -= 1;
    if (q < (depth - 1) * NMB) {
        off = (int)(L.grad_off + (L.grad_layer_tile(depth - 1 - q / NMB) + q % NMB) * tb);
        ks = NKB;
        stride = NMB * tb;
        return;
    }
    q -= (depth - 1) * NMB;
    off = (int)(L.grad_off + (L.grad_layer_tile(0) + q) * tb);
    ks = NKB;
    stride = kGradRowBlocks0 * tb;
}

// Per-launch tables in LDS: for every network, its blob address, depth and phase program.
struct NetTable {
    uint64_t blob[kMaxNets];
    int depth[kMaxNets];
    int nphase[kMaxNets];
    int ph[kMaxNets][kMaxPhases][3];   // offset, stride, tiles
};

// One wave's share of a phase: nothing is held in registers, the loads write LDS directly;
// only whether the phase exists is kept.
template <int W>
struct Stage {
    static constexpr int kMax = (W / 16 + 1 + Geo<W>::kWaves - 1) / Geo<W>::kWaves;
    int cnt;   // wave-uniform
};

// Where one phase's tiles come from: global address of its first tile, byte stride between
// tiles, tile count, and whether the phase exists (wave-uniform values).
struct Desc {
    uint64_t addr;
    int stride, ks, live;
};

// The phase pipeline of a workgroup: the current tile's network and phase, the next tile's
// network (-1: none) with both networks' phase counts and blob addresses, the stage in use,
// and the descriptor of the phase two ahead of the current one (looked up one phase early,
// so a phase starts its fetch without waiting on the table).
struct Pipe {
    int cur, q, nxt;
    int stage;   // 0 .. stages - 1
    int np_cur, np_nxt;
    uint64_t blob_cur, blob_nxt;
    Desc d2;
};

__device__ inline uint64_t uniform_u64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline void pipe_tiles(Pipe &pp, const NetTable *tab, int cur, int nxt) {
    pp.cur = cur;
    pp.nxt = nxt;
    pp.q = 0;
    pp.np_cur = __builtin_amdgcn_readfirstlane(tab->nphase[cur]);
    pp.blob_cur = uniform_u64(tab->blob[cur]);
    const int nn = nxt >= 0 ? nxt : cur;
    pp.np_nxt = nxt >= 0 ? __builtin_amdgcn_readfirstlane(tab->nphase[nn]) : 0;
    pp.blob_nxt = uniform_u64(tab->blob[nn]);
}

// Phase `ahead` phases after the current one, in two steps: the table read is issued by
// desc_issue and turned into wave-uniform values by desc_finish (after a wait that the
// caller has anyway).
struct DescRaw {
    int off, stride, ks;   // per lane (all lanes read the same entry)
    uint64_t blob;
    int live;
};

__device__ inline DescRaw desc_issue(const NetTable *tab, const Pipe &pp, int ahead) {
    int q = pp.q + ahead;
    const bool nx = q >= pp.np_cur;
    const int net = nx ? pp.nxt : pp.cur;
    q = nx ? q - pp.np_cur : q;
    const int np = nx ? pp.np_nxt : pp.np_cur;
    DescRaw r;
    r.live = net >= 0 && q < np;
    r.blob = nx ? pp.blob_nxt : pp.blob_cur;
    const int *e = tab->ph[r.live ? net : 0][r.live ? q : 0];
    r.off = e[0];
    r.stride = e[1];
    r.ks = e[2];
    return r;
}

__device__ inline Desc desc_finish(const DescRaw &r) {
    Desc d;
    d.live = r.live;
    const int off = __builtin_amdgcn_readfirstlane(r.off);
    d.stride = __builtin_amdgcn_readfirstlane(r.stride);
    d.ks = __builtin_amdgcn_readfirstlane(r.ks);
    d.addr = r.blob + (uint64_t)(int64_t)off;
    return d;
}

template <int W>
__device__ inline lds_u8 *stage_ptr(lds_u8 *ring, int st) {
    return ring + st * (W / 16 + 1) * 1024;
}

// Fetches this wave's share of the phase that `d` describes straight into its LDS stage
// (buffer loads that write LDS, 16 bytes per lane: one instruction moves one whole 1 KiB tile,
// lane-major, which is the tile's layout).  Branch-free over the share: slot i takes tile
// min(i, ks - 1), so extra loads of a short phase rewrite its last tile with the same bytes.
// The buffer form (not the global one) keeps the compiler's waits for the ring's LDS reads
// exact: after a global load into LDS it waits for every outstanding LDS read instead of only
// the one an MFMA needs.  The resource covers exactly the phase's tiles.
template <int W>
__device__ inline void stage_fetch(Stage<W> &sg, const Desc &d, lds_u8 *stage, int wave, int lane) {
    sg.cnt = d.live;
    if (!sg.cnt) return;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)d.addr, 0, (d.ks - 1) * d.stride + 1024, 0x00020000);
#pragma unroll
    for (int j = 0; j < Stage<W>::kMax; ++j) {
        const int i = min(wave + Geo<W>::kWaves * j, d.ks - 1);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)(stage + i * 1024), 16,
                                                 i * d.stride + lane * 16, 0, 0, 0);
    }
}

// The compiler does not track the LDS writes of the buffer loads: wait for them explicitly
// (vmcnt(0), other counters left alone) before the barrier that publishes the stage.
__device__ inline void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Start of a phase: issue this wave's loads of the phase two ahead (into the stage that the
// phase two back used) and the table read for the phase after that.
template <int W>
__device__ inline DescRaw phase_begin(Stage<W> &sg, lds_u8 *ring, const NetTable *tab, const Pipe &pp, int wave,
                                      int lane) {
    stage_fetch<W>(sg, pp.d2, stage_ptr<W>(ring, (pp.stage + 2) % Ring<W>::kStages), wave, lane);
    if constexpr (Ring<W>::kPair) return desc_issue(tab, pp, 3);
    return DescRaw{};   // single mode reads the table at the end of the phase (fewer live registers)
}

// End of a phase.  With `bar` the barrier waits for this wave's loads and publishes the next
// stages; in pair mode only the second phase of a pair (or a lone phase) has one, so every
// phase is still separated by a barrier from the phase two before it, whose stage its loads
// overwrite, and its own stage was loaded and published before it starts.
template <int W>
__device__ inline void phase_end(const DescRaw &nd_begin, const NetTable *tab, Pipe &pp, bool bar) {
    const DescRaw nd = Ring<W>::kPair ? nd_begin : desc_issue(tab, pp, 3);
    if (bar) {
        stage_wait();
        __syncthreads();
    }
    pp.d2 = desc_finish(nd);
    pp.stage = pp.stage == Ring<W>::kStages - 1 ? 0 : pp.stage + 1;
    ++pp.q;
}

__device__ inline bf16x8 lds_tile(const lds_u8 *stage, int i, int lane) {
    return *reinterpret_cast<const __attribute__((address_space(3))) bf16x8 *>(stage + i * 1024 + lane * 16);
}

// A tiles in flight: the first kAR tiles of the current phase are loaded during the
// previous phase (its stage was published one barrier earlier), so a phase starts without
// waiting on LDS, and inside a phase each tile is read kAR MFMA steps before its use.
constexpr int kAR = 4;
struct ARing {
    bf16x8 r[kAR];
};

// One phase's MFMA chain: KS K-blocks from the stage (the last one the bias block when
// kBias).  kHaveFirst: the ring holds tiles 0 .. kAR - 1 already (else they are read here);
// kNext: the last kAR steps load the next phase's first tiles (its stage is published).
template <int W, int KS, bool kBias, bool kHaveFirst = true, bool kNext = true>
__device__ __attribute__((always_inline)) inline void phase_mfma(const lds_u8 *st, const lds_u8 *st_next, ARing &ar,
                                                                 const bf16x8 (&bin)[W / 16][Geo<W>::kNB],
                                                                 f32x16 (&acc)[Geo<W>::kNB], int lane, int h) {
    constexpr int kNB = Geo<W>::kNB;
    constexpr int KIN = KS - (kBias ? 1 : 0);
    static_assert(KS >= kAR, "every phase has at least kAR tiles");
    const bf16x8 one = bias_operand(h);
    if constexpr (!kHaveFirst) {
#pragma unroll
        for (int j = 0; j < kAR; ++j) ar.r[j] = lds_tile(st, j, lane);
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 a = ar.r[ks % kAR];
        if (ks + kAR < KS) ar.r[ks % kAR] = lds_tile(st, ks + kAR, lane);
        else if (kNext) ar.r[ks % kAR] = lds_tile(st_next, ks + kAR - KS, lane);
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const bf16x8 b = (kBias && ks == KIN) ? one : bin[ks < KIN ? ks : 0][nb];
            acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, ks == 0 ? f32x16{} : acc[nb], 0, 0, 0);
        }
    }
    if constexpr (kNext) {   // the next phase's tile j landed in slot (KS + j) % kAR: restore the order
        ARing t = ar;
#pragma unroll
        for (int j = 0; j < kAR; ++j) ar.r[j] = t.r[(KS + j) % kAR];
    }
}

template <int W>
__device__ inline const lds_u8 *cur_stage(lds_u8 *ring, const Pipe &pp) {
    return stage_ptr<W>(ring, pp.stage);
}
template <int W>
__device__ inline const lds_u8 *nxt_stage(lds_u8 *ring, const Pipe &pp) {
    return stage_ptr<W>(ring, pp.stage == Ring<W>::kStages - 1 ? 0 : pp.stage + 1);
}

template <int W>
__device__ inline void relu_mask_out(const f32x16 &y, int l, int mb, int nb, bf16x8 (&bout)[W / 16][Geo<W>::kNB],
                                     uint16_t *wmask, int lane, bool grad) {
    constexpr int NMB = W / 32, kNB = Geo<W>::kNB;
    if (grad) {
        uint32_t bits = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) bits |= (y[j] > 0.f ? 1u : 0u) << j;
        wmask[((l * NMB + mb) * kNB + nb) * 64 + lane] = (uint16_t)bits;
    }
    relu_tile_to_bf16(y, mb, nb, bout);
    // keep the conversion in this phase (interleaved with its MFMA chain) rather than sunk to
    // the end of the layer, where it would hold every M-block's accumulators live
    asm volatile("" : "+v"(bout[2 * mb][nb]), "+v"(bout[2 * mb + 1][nb]));
}

// Forward layer l (all its M-blocks): bin -> bout with ReLU; masks to LDS for gradients.
template <int W, int KIN, bool kGrad>
__device__ __attribute__((always_inline)) inline void fwd_layer(lds_u8 *ring, const NetTable *tab, Pipe &pp, ARing &ar, int l,
                                                                const bf16x8 (&bin)[W / 16][Geo<W>::kNB],
                                                                bf16x8 (&bout)[W / 16][Geo<W>::kNB], uint16_t *wmask,
                                                                int wave, int lane, int h) {
    constexpr int NMB = W / 32, NKB = W / 16, kNB = Geo<W>::kNB;
    constexpr bool kBias = KIN == NKB;
    f32x16 acc[2][kNB];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
        Stage<W> sg;
        const DescRaw nd = phase_begin<W>(sg, ring, tab, pp, wave, lane);
        if (!Ring<W>::kPair)
            phase_mfma<W, KIN + (kBias ? 1 : 0), kBias>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, bin,
                                                        acc[mb & 1], lane, h);
        else if (mb & 1)   // second of a pair (the loop is unrolled: mb is a constant here)
            phase_mfma<W, KIN + (kBias ? 1 : 0), kBias, true, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar,
                                                                     bin, acc[mb & 1], lane, h);
        else
            phase_mfma<W, KIN + (kBias ? 1 : 0), kBias, false, true>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar,
                                                                     bin, acc[mb & 1], lane, h);
        if (mb > 0) {
#pragma unroll
            for (int nb = 0; nb < kNB; ++nb) relu_mask_out<W>(acc[(mb - 1) & 1][nb], l, mb - 1, nb, bout, wmask, lane, kGrad);
        }
        phase_end<W>(nd, tab, pp, !Ring<W>::kPair || (mb & 1));
    }
#pragma unroll
    for (int nb = 0; nb < kNB; ++nb) relu_mask_out<W>(acc[(NMB - 1) & 1][nb], l, NMB - 1, nb, bout, wmask, lane, kGrad);
}

// Masked adjoint tile -> bf16 B operands of the next transposed product.
template <int W>
__device__ inline void masked_tile_to_bf16(const f32x16 &y, uint32_t bits, int mb, int nb,
                                           bf16x8 (&b)[W / 16][Geo<W>::kNB]) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j)   // bit j sign-extended to 0 or all ones, then AND: y_j or +0
        v[j] = __uint_as_float(__float_as_uint(y[j]) & (uint32_t)__builtin_amdgcn_sbfe((int)bits, j, 1));
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < 8; ++s) b[2 * mb + c][nb][s] = (__bf16)v[8 * c + s];
    asm volatile("" : "+v"(b[2 * mb][nb]), "+v"(b[2 * mb + 1][nb]));
}

// Transposed hidden layer l (rows: its inputs): adjoint operands of layer l's outputs ->
// masked adjoint operands of layer l - 1's outputs.
// Phase of a wave that has nothing to compute: the ring still moves on to the next phase's
// first tiles, and the caller still takes part in the fetch and the barrier.
template <int W>
__device__ __attribute__((always_inline)) inline void phase_skip(const lds_u8 *st_next, ARing &ar, int lane) {
#pragma unroll
    for (int j = 0; j < kAR; ++j) ar.r[j] = lds_tile(st_next, j, lane);
}

template <int W>
__device__ __attribute__((always_inline)) inline void bwd_layer(lds_u8 *ring, const NetTable *tab, Pipe &pp, ARing &ar, int l,
                                                                const bf16x8 (&bin)[W / 16][Geo<W>::kNB],
                                                                bf16x8 (&bout)[W / 16][Geo<W>::kNB],
                                                                const uint16_t *wmask, int wave, int lane, int h) {
    constexpr int NMB = W / 32, NKB = W / 16, kNB = Geo<W>::kNB;
    f32x16 acc[2][kNB];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) {
        Stage<W> sg;
        const DescRaw nd = phase_begin<W>(sg, ring, tab, pp, wave, lane);
        if (!Ring<W>::kPair)
            phase_mfma<W, NKB, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, bin, acc[mb & 1], lane, h);
        else if (mb & 1)
            phase_mfma<W, NKB, false, true, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, bin, acc[mb & 1],
                                                   lane, h);
        else
            phase_mfma<W, NKB, false, false, true>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, bin, acc[mb & 1],
                                                   lane, h);
        if (mb > 0) {
#pragma unroll
            for (int nb = 0; nb < kNB; ++nb)
                masked_tile_to_bf16<W>(acc[(mb - 1) & 1][nb], wmask[(((l - 1) * NMB + mb - 1) * kNB + nb) * 64 + lane],
                                       mb - 1, nb, bout);
        }
        phase_end<W>(nd, tab, pp, !Ring<W>::kPair || (mb & 1));
    }
#pragma unroll
    for (int nb = 0; nb < kNB; ++nb)
        masked_tile_to_bf16<W>(acc[(NMB - 1) & 1][nb], wmask[(((l - 1) * NMB + NMB - 1) * kNB + nb) * 64 + lane],
                               NMB - 1, nb, bout);
}

// Network and ray range of workgroup tile t (constant indices into the argument arrays: a
// runtime index would copy them to scratch).
struct TileWork {
    int net;
    int64_t base, end;   // rays [base, min(base + 256, end))
};

__device__ inline TileWork tile_work(const GradArgs &a, int64_t t, const int64_t (&pre)[kMaxNets + 1], int nk,
                                     int64_t count) {
    TileWork w;
    const bool multi = a.n_nets > 0;
    int k = 0;
#pragma unroll
    for (int i = 1; i < kMaxNets; ++i)
        if (i < nk && t >= pre[i]) k = i;
    int64_t lo = 0, cnt = count, pk = 0;
    if (multi) {
        lo = a.seg_offset[k];
        cnt = a.seg_count[k];
    }
#pragma unroll
    for (int i = 0; i < kMaxNets; ++i)
        if (i == k) pk = pre[i];
    w.net = k;
    w.end = lo + cnt;
    w.base = lo + (t - pk) * kRaysPerTile;
    return w;
}

template <int W, bool kGrad>
__global__ __launch_bounds__(Geo<W>::kWaves * 64, 2) void stream_kernel(GradArgs a) {
    constexpr int NMB = W / 32, NKB = W / 16, K0 = layer0_kblocks(kBF16);
    constexpr int kWaves = Geo<W>::kWaves, kNB = Geo<W>::kNB;
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = lane >> 5, col = lane & 31;
    const bool multi = a.n_nets > 0;
    const int nk = multi ? a.n_nets : 1;
    const int64_t n = a.n;
    const int64_t count = a.count_dev ? min<int64_t>(*a.count_dev, n) : n;
    const int dmax = a.depth;

    // LDS: weight ring | network tables | ReLU masks [wave][depth][NMB][kNB][64] | head rows
    lds_u8 *ring = (lds_u8 *)smem;
    NetTable *tab = reinterpret_cast<NetTable *>(smem + Ring<W>::kStages * (NKB + 1) * 1024);
    uint16_t *s_mask = reinterpret_cast<uint16_t *>(tab + 1);
    float *s_head = reinterpret_cast<float *>(s_mask + (kGrad ? kWaves * dmax * NMB * kNB * 64 : 0));
    uint16_t *wmask = s_mask + wave * dmax * NMB * kNB * 64;
#pragma unroll
    for (int k = 0; k < kMaxNets; ++k) {
        if (k >= nk) break;
        const uint8_t *blob = multi ? a.blobs[k] : a.blob;
        const int depth = multi ? a.depths[k] : a.depth;
        const int np = phases_of<W>(depth, kGrad);
        if (threadIdx.x == 0) {
            tab->blob[k] = (uint64_t)blob;
            tab->depth[k] = depth;
            tab->nphase[k] = np;
        }
        for (int q = threadIdx.x; q < np; q += blockDim.x) {
            int off, stride, ks;
            phase_entry<W>(depth, q, off, stride, ks);
            tab->ph[k][q][0] = off;
            tab->ph[k][q][1] = stride;
            tab->ph[k][q][2] = ks;
        }
        if constexpr (kGrad) {
            const NetLayout L = make_layout(W, depth, kBF16);
            const float *src = reinterpret_cast<const float *>(blob + L.head_rows_off);
            for (int i = threadIdx.x; i < 2 * W; i += blockDim.x) s_head[k * 2 * W + i] = src[i];
        }
    }
    __syncthreads();

    int64_t pre[kMaxNets + 1];
    pre[0] = 0;
#pragma unroll
    for (int k = 0; k < kMaxNets; ++k) {
        const int64_t cnt = k < nk ? (multi ? (int64_t)a.seg_count[k] : count) : 0;
        pre[k + 1] = pre[k] + (cnt + kRaysPerTile - 1) / kRaysPerTile;
    }
    const int64_t ntile = pre[kMaxNets];
    int64_t t = blockIdx.x;
    if (t >= ntile) return;   // the whole workgroup: no barrier is left half-reached

    Pipe pp;
    TileWork cw = tile_work(a, t, pre, nk, count);
    pipe_tiles(pp, tab, cw.net, t + gridDim.x < ntile ? tile_work(a, t + gridDim.x, pre, nk, count).net : -1);
    pp.stage = 0;
    {   // prologue: phases 0 and 1 into stages 0 and 1
        Stage<W> s0, s1;
        stage_fetch<W>(s0, desc_finish(desc_issue(tab, pp, 0)), stage_ptr<W>(ring, 0), wave, lane);
        stage_fetch<W>(s1, desc_finish(desc_issue(tab, pp, 1)), stage_ptr<W>(ring, 1), wave, lane);
        pp.d2 = desc_finish(desc_issue(tab, pp, 2));
        stage_wait();
        __syncthreads();
    }
    ARing ar;   // in pair mode the first phase follows a barrier and fills it itself
    if constexpr (!Ring<W>::kPair) {
#pragma unroll
        for (int j = 0; j < kAR; ++j) ar.r[j] = lds_tile(stage_ptr<W>(ring, 0), j, lane);
    }

    for (;;) {
        const int depth = __builtin_amdgcn_readfirstlane(tab->depth[pp.cur]);
        const float *head = s_head + pp.cur * 2 * W;
        bf16x8 b0[NKB][kNB], b1[NKB][kNB];
        float v[kNB][kInRaw];
        bool valid[kNB];
        // ---- encoding -> layer-0 operands (bias in two feature slots of lane half 1)
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t r = cw.base + (wave * kNB + nb) * 32 + col;
            valid[nb] = r < cw.end;
#pragma unroll
            for (int j = 0; j < kInRaw; ++j) v[nb][j] = valid[nb] ? a.rays[(int64_t)j * n + r] : 0.f;
            float feat[kSlotsPerHalf];
            encode_var<false>(h ? v[nb][3] : v[nb][0], feat);
            encode_var<false>(h ? v[nb][4] : v[nb][1], feat + kFeatPerVar);
            encode_var<false>(h ? 0.f : v[nb][2], feat + 2 * kFeatPerVar);
            feat[kSlotsPerHalf - 1] = 0.f;
            feat[kBiasSlot0] = h ? 1.f : feat[kBiasSlot0];
            feat[kBiasSlot1] = h ? 1.f : 0.f;
#pragma unroll
            for (int kb = 0; kb < K0; ++kb)
#pragma unroll
                for (int s = 0; s < 8; ++s) b0[kb][nb][s] = (__bf16)feat[kb * 8 + s];
        }
        // ---- forward: layer 0 into b1, then hidden layers alternating; the last output ends in b1
        fwd_layer<W, K0, kGrad>(ring, tab, pp, ar, 0, b0, b1, wmask, wave, lane, h);
        int l = 1;
        if ((depth - 1) % 2 == 1) {   // odd count of hidden layers: one step first, then pairs
            fwd_layer<W, NKB, kGrad>(ring, tab, pp, ar, 1, b1, b0, wmask, wave, lane, h);
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                for (int nb = 0; nb < kNB; ++nb) b1[kb][nb] = b0[kb][nb];
            l = 2;
        }
        for (; l + 1 < depth; l += 2) {
            fwd_layer<W, NKB, kGrad>(ring, tab, pp, ar, l, b1, b0, wmask, wave, lane, h);
            fwd_layer<W, NKB, kGrad>(ring, tab, pp, ar, l + 1, b0, b1, wmask, wave, lane, h);
        }
        // ---- head: logit and distance in rows 0 and 1 of lane half 0
        f32x16 hacc[kNB];
        {
            Stage<W> sg;   // in pair mode a lone phase
            const DescRaw nd = phase_begin<W>(sg, ring, tab, pp, wave, lane);
            if constexpr (Ring<W>::kPair)
                phase_mfma<W, NKB + 1, true, false, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, b1, hacc,
                                                           lane, h);
            else
                phase_mfma<W, NKB + 1, true>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, b1, hacc, lane, h);
            phase_end<W>(nd, tab, pp, true);
        }
        float gl[kNB], gd[kNB];
        bool any_hit = false;   // some ray of this wave has logit > 0
#pragma unroll
        for (int nb = 0; nb < kNB; ++nb) {
            const int64_t r = cw.base + (wave * kNB + nb) * 32 + col;
            // rows 2 and 3 hold the bf16 remainders of the head rows 0 and 1
            const float z = __shfl(hacc[nb][0] + hacc[nb][2], col), dd = __shfl(hacc[nb][1] + hacc[nb][3], col);
            any_hit |= __ballot(valid[nb] && z > 0.f) != 0;
            float *dst = h ? a.dist_out : a.logit_out;
            if (valid[nb] && dst) dst[r] = h ? dd : z;
            gl[nb] = (kGrad && valid[nb] && a.g_logit_in) ? a.g_logit_in[r] : 0.f;
            gd[nb] = (kGrad && valid[nb] && a.g_dist_in) ? a.g_dist_in[r] : 0.f;
        }
        if constexpr (kGrad) {
            // with grad_hits_only a wave whose rays all miss skips the reverse sweep: it only
            // walks the phases (fetch, ring, barrier) and writes no gradient
            const bool active = !a.grad_hits_only || any_hit;   // wave-uniform
            if (!active) {
                // (the barriers of the active waves: in pair mode pairs in the hidden layers, then
                // a pair and a lone phase in the transposed layer 0)
                const int nh = (depth - 1) * NMB, nbwd = nh + kGradRowBlocks0;
                for (int i = 0; i < nbwd; ++i) {
                    Stage<W> sg;
                    const DescRaw nd = phase_begin<W>(sg, ring, tab, pp, wave, lane);
                    if constexpr (!Ring<W>::kPair) phase_skip<W>(nxt_stage<W>(ring, pp), ar, lane);
                    phase_end<W>(nd, tab, pp, !Ring<W>::kPair || (i < nh ? (i & 1) == 1 : i != nh));
                }
            } else {
            // ---- seed: adjoint of the last hidden layer = head rows x seeds, masked -> b0
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) {
                f32x16 w0, w1;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const f32x4 a4 = *reinterpret_cast<const f32x4 *>(head + mb * 32 + 8 * g + 4 * h);
                    const f32x4 b4 = *reinterpret_cast<const f32x4 *>(head + W + mb * 32 + 8 * g + 4 * h);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        w0[4 * g + i] = a4[i];
                        w1[4 * g + i] = b4[i];
                    }
                }
#pragma unroll
                for (int nb = 0; nb < kNB; ++nb) {
                    f32x16 y;
#pragma unroll
                    for (int j = 0; j < 16; ++j) y[j] = fmaf(gl[nb], w0[j], gd[nb] * w1[j]);
                    masked_tile_to_bf16<W>(y, wmask[(((depth - 1) * NMB + mb) * kNB + nb) * 64 + lane], mb, nb, b0);
                }
            }
            // ---- transposed hidden layers from the top; the last adjoint ends in b0
            int lb = depth - 1;
            if (lb % 2 == 1) {
                bwd_layer<W>(ring, tab, pp, ar, lb, b0, b1, wmask, wave, lane, h);
#pragma unroll
                for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                    for (int nb = 0; nb < kNB; ++nb) b0[kb][nb] = b1[kb][nb];
                --lb;
            }
            for (; lb >= 2; lb -= 2) {
                bwd_layer<W>(ring, tab, pp, ar, lb, b0, b1, wmask, wave, lane, h);
                bwd_layer<W>(ring, tab, pp, ar, lb - 1, b1, b0, wmask, wave, lane, h);
            }
            // ---- transposed layer 0: adjoints of this lane's feature slots
            f32x16 acc0[kGradRowBlocks0][kNB];
#pragma unroll
            for (int mb = 0; mb < kGradRowBlocks0; ++mb) {   // in pair mode: a pair, then a lone phase
                static_assert(kGradRowBlocks0 == 3, "transposed layer 0: three M-blocks");
                Stage<W> sg;
                const DescRaw nd = phase_begin<W>(sg, ring, tab, pp, wave, lane);
                if (!Ring<W>::kPair)
                    phase_mfma<W, NKB, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, b0, acc0[mb], lane, h);
                else if (mb == 0)
                    phase_mfma<W, NKB, false, false, true>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, b0, acc0[mb],
                                                           lane, h);
                else if (mb == 1)
                    phase_mfma<W, NKB, false, true, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, b0, acc0[mb],
                                                           lane, h);
                else
                    phase_mfma<W, NKB, false, false, false>(cur_stage<W>(ring, pp), nxt_stage<W>(ring, pp), ar, b0,
                                                            acc0[mb], lane, h);
                phase_end<W>(nd, tab, pp, !Ring<W>::kPair || mb != 0);
            }
            // ---- chain rule through the Fourier features
#pragma unroll
            for (int nb = 0; nb < kNB; ++nb) {
                const int64_t r = cw.base + (wave * kNB + nb) * 32 + col;
#pragma unroll
                for (int var = 0; var < 3; ++var) {
                    if (h == 1 && var == 2) continue;
                    float f[kFeatPerVar];
                    const float x = h ? v[nb][3 + var] : v[nb][var];
                    encode_var<false>(x, f);
                    float g = acc0[(var * kFeatPerVar) / 16][nb][(var * kFeatPerVar) % 16];
#pragma unroll
                    for (int k = 0; k < kNFreq; ++k) {
                        const int fs = var * kFeatPerVar + 1 + k, fc = var * kFeatPerVar + 1 + kNFreq + k;
                        const float gs = acc0[fs / 16][nb][fs % 16], gc = acc0[fc / 16][nb][fc % 16];
                        g = fmaf((float)(1 << k), gs * f[1 + kNFreq + k] - gc * f[1 + k], g);
                    }
                    if (valid[nb] && a.g_rays) a.g_rays[(int64_t)(h ? 3 + var : var) * n + r] = g;
                }
            }
            }   // active
        }
        // ---- next workgroup tile
        t += gridDim.x;
        if (t >= ntile) break;
        cw = tile_work(a, t, pre, nk, count);
        pipe_tiles(pp, tab, cw.net, t + gridDim.x < ntile ? tile_work(a, t + gridDim.x, pre, nk, count).net : -1);
    }
}

int cu_count_stream() {
    static int cus = 0;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    });
    return cus;
}

template <int W, bool kGrad>
ddf_status launch_stream(const GradArgs &args, hipStream_t s) {
    auto kern = stream_kernel<W, kGrad>;
    static std::once_flag once;
    std::call_once(once, [&] { (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxStreamLds); });
    const int nk = args.n_nets > 0 ? args.n_nets : 1;
    DDF_REQUIRE(args.depth >= 1 && args.depth <= 8 && nk <= kMaxNets, DDF_ERR_UNSUPPORTED,
                "streamed network kernel: depth 1..8 and at most %d networks", kMaxNets);
    const size_t lds = stream_lds_bytes(W, args.depth, nk, kGrad);
    DDF_REQUIRE(lds <= (size_t)kMaxStreamLds, DDF_ERR_UNSUPPORTED, "network too deep for the streamed kernel");
    // persistent: one workgroup of eight waves per CU at width 256; at width 128 one or two
    // workgroups of four waves (a tuning knob; two only when their LDS fits)
    const int per_cu = W == 128 && lds * 2 <= (size_t)kMaxStreamLds ? tuning(DDF_TUNE_STREAM_WG_PER_CU) : 1;
    const int64_t tiles_hint = (args.n + kRaysPerTile - 1) / kRaysPerTile + nk;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(tiles_hint, (int64_t)cu_count_stream() * per_cu));
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(Geo<W>::kWaves * 64), lds, s, args);
    return launch_status("ddf streamed network kernel");
}

}  // namespace

size_t stream_lds_bytes(int width, int depth, int n_nets, bool grad) {
    const int nmb = width / 32, nkb = width / 16;
    const int waves = width == 256 ? Geo<256>::kWaves : Geo<128>::kWaves;
    const int nb = width == 256 ? Geo<256>::kNB : Geo<128>::kNB;
    const int stages = width == 256 ? Ring<256>::kStages : Ring<128>::kStages;
    size_t b = (size_t)stages * (nkb + 1) * 1024 + sizeof(NetTable);
    if (grad) b += (size_t)waves * depth * nmb * nb * 64 * 2 + (size_t)n_nets * 2 * width * 4;
    return b;
}

// bf16 networks of width 128 or 256; args.depth is the largest depth of the launch.
ddf_status stream_dispatch(int width, const GradArgs &args, hipStream_t s) {
    const bool grad = !args.forward_only;
    if (width == 256) return grad ? launch_stream<256, true>(args, s) : launch_stream<256, false>(args, s);
    return grad ? launch_stream<128, true>(args, s) : launch_stream<128, false>(args, s);
}

}  // namespace ddf
