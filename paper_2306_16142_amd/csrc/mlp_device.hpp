// Device building blocks of the network kernels: Fourier encoding, MFMA wrappers and
// operand loads (operand numbering in mlp_layout.hpp).
#pragma once
#include "common.hpp"
#include "mlp_layout.hpp"

namespace ddf {

constexpr float kFp8Max = 448.0f;

// ------------------------------------------------------------------------------ encoding
// sin and cos of one float32 argument of moderate size (|v| <= kSinCosFastMax), written from
// the mathematics: Cody-Waite reduction r = v - j pi/2, j = nearest integer to v 2/pi, with
// pi/2 split into three float32 parts C1 + C2 + C3 (C1 = fl(pi/2), C2 = fl(pi/2 - C1),
// C3 = fl(pi/2 - C1 - C2)) applied by fused multiply-adds; the Taylor series of sin to r^9
// and of cos to r^10 on |r| <= pi/4 (truncation below 2e-9); the quadrant j mod 4 picks and
// signs the pair.  Absolute error below 7.1e-8 (1.2 float32 ulp of 1) over the range.  A
// wavefront holding any larger, infinite or NaN argument calls sincosf for all its lanes, so
// the general reduction costs nothing on the usual inputs (coordinates and angles).
constexpr float kSinCosFastMax = 1024.f;

__device__ inline void sincos_moderate(float v, float &s, float &c) {
    if (__builtin_expect(__any(!(fabsf(v) <= kSinCosFastMax)), 0)) {
        sincosf(v, &s, &c);
        return;
    }
    const float j = __builtin_rintf(v * 0x1.45f306p-1f);   // 2/pi
    float r = fmaf(-j, 0x1.921fb6p+0f, v);
    r = fmaf(-j, -0x1.777a5cp-25f, r);
    r = fmaf(-j, -0x1.ee59dap-50f, r);
    const float r2 = r * r;
    float ps = fmaf(r2, 0x1.71de3ap-19f, -0x1.a01a02p-13f);   // 1/9!, -1/7!
    ps = fmaf(r2, ps, 0x1.111112p-7f);                         // 1/5!
    ps = fmaf(r2, ps, -0x1.555556p-3f);                        // -1/3!
    const float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -0x1.27e4fcp-22f, 0x1.a01a02p-16f);    // -1/10!, 1/8!
    pc = fmaf(r2, pc, -0x1.6c16c2p-10f);                       // -1/6!
    pc = fmaf(r2, pc, 0x1.555556p-5f);                         // 1/4!
    pc = fmaf(r2, pc, -0.5f);
    const float cr = fmaf(r2, pc, 1.0f);
    const int q = (int)j;
    const bool odd = q & 1;
    const float so = odd ? cr : sr, co = odd ? sr : cr;
    s = __uint_as_float(__float_as_uint(so) ^ ((uint32_t)(q & 2) << 30));
    c = __uint_as_float(__float_as_uint(co) ^ ((uint32_t)((q + 1) & 2) << 30));
}

// sin and cos of v from the hardware's sine and cosine (whose argument is in turns), for
// features that are rounded to e4m3 (3 mantissa bits): the units' error, amplified 32x by the
// double-angle recurrence at the top frequency, stays far below one e4m3 step.  A wavefront
// holding any argument beyond kSinCosFastMax (or infinite or NaN) calls sincosf.
__device__ inline void sincos_hw(float v, float &s, float &c) {
    if (__builtin_expect(__any(!(fabsf(v) <= kSinCosFastMax)), 0)) {
        sincosf(v, &s, &c);
        return;
    }
    const float turns = v * 0x1.45f306p-3f;   // 1 / (2 pi)
    s = __builtin_amdgcn_sinf(turns);
    c = __builtin_amdgcn_cosf(turns);
}

// Features of one variable: raw, sin(2^k v), cos(2^k v), k = 0..5.  In float32 mode every
// frequency calls sincosf (arguments 2^k v are exact); in reduced precision the base pair
// comes from sincos_moderate (bf16) or the hardware units (kHw: fp8) and the higher
// frequencies follow the double-angle recurrence.  (The hardware sine was tried for the bf16
// base frequency: its error, amplified 32x by the recurrence, flipped visibly more bf16
// roundings than float32 rounding does.)
template <bool kExact, bool kHw = false>
__device__ inline void encode_var(float v, float *f) {
    f[0] = v;
    float s, c;
    if constexpr (kExact) sincosf(v, &s, &c);
    else if constexpr (kHw) sincos_hw(v, s, c);
    else sincos_moderate(v, s, c);
    f[1] = s;
    f[1 + kNFreq] = c;
#pragma unroll
    for (int k = 1; k < kNFreq; ++k) {
        if constexpr (kExact) {
            sincosf(v * (float)(1 << k), &s, &c);
        } else {
            const float s2 = 2.f * s * c;
            const float c2 = 1.f - 2.f * s * s;
            s = s2;
            c = c2;
        }
        f[1 + k] = s;
        f[1 + kNFreq + k] = c;
    }
}

// ------------------------------------------------------------------------------ forward
template <int P>
struct OpOf;
template <>
struct OpOf<kBF16> {
    using T = bf16x8;
};
template <>
struct OpOf<kFP8> {
    using T = i32x8;
};
template <>
struct OpOf<kFP32> {
    using T = float;
};

template <int P>
__device__ inline f32x16 mfma(typename OpOf<P>::T a, typename OpOf<P>::T b, f32x16 c) {
    if constexpr (P == kBF16) return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    else if constexpr (P == kFP8) return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    else return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// A operand of one lane.  An fp8 tile (32 bytes per lane) is stored as two 1 KiB halves,
// bytes 0-15 of every lane then bytes 16-31 of every lane, so that each of the two 16-byte
// reads covers consecutive addresses across the lanes (free of LDS bank conflicts).
template <int P>
__device__ inline typename OpOf<P>::T load_a(const uint8_t *src, int64_t tile, int lane) {
    using Op = typename OpOf<P>::T;
    if constexpr (P == kFP8) {
        const uint8_t *p = src + tile * tile_bytes(P) + (int64_t)lane * 16;
        const i32x4 lo = *reinterpret_cast<const i32x4 *>(p), hi = *reinterpret_cast<const i32x4 *>(p + 1024);
        return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    } else {
        const uint8_t *p = src + tile * tile_bytes(P) + (int64_t)lane * (tile_bytes(P) / 64);
        return *reinterpret_cast<const Op *>(p);
    }
}

// Packs 4 non-negative floats (already clamped to the e4m3 range) into one dword.
__device__ inline int pack_fp8x4(float a, float b, float c, float d) {
    // the first conversion writes the low half and keeps the high half of its third
    // operand, which the second conversion overwrites: any register will do there
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, __builtin_bit_cast(int, a), false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}


__device__ inline uint16_t bf16_bits(float x) {
    __bf16 b = (__bf16)x;   // round to nearest even
    return __builtin_bit_cast(uint16_t, b);
}

__device__ inline uint8_t fp8_bits(float x) {
    x = __builtin_amdgcn_fmed3f(x, -kFp8Max, kFp8Max);   // the conversion does not saturate
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
}

// B operand of the bf16 bias K-block: 1.0 in slots 0 and 1 of lane half 0.
__device__ inline bf16x8 bias_operand(int h) {
    bf16x8 v;
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = (__bf16)((h == 0 && s < 2) ? 1.0f : 0.0f);
    return v;
}

// ReLU of two floats rounded to a packed bf16 pair.  Read as 16-bit integers, every bf16
// with the sign bit set (-0 included) is negative and every other one non-negative, so a
// signed integer max with 0 is the ReLU; rounding to bf16 keeps the sign, so ReLU after
// rounding equals rounding after ReLU.  One packed conversion and one packed integer max
// per two values.
__device__ inline uint32_t relu_pk_bf16(float a, float b) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = __builtin_convertvector((f32x2){a, b}, bf16x2);   // round to nearest even
    const s16x2 m = __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), (s16x2){0, 0});
    return __builtin_bit_cast(uint32_t, m);
}

// ReLU of one accumulator tile (M-block mb) into the next product's bf16 B operands.
template <int NKB, int NB>
__device__ inline void relu_tile_to_bf16(const f32x16 &y, int mb, int nb, bf16x8 (&b)[NKB][NB]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        u32x4 w;
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = relu_pk_bf16(y[8 * c + 2 * q], y[8 * c + 2 * q + 1]);
        b[2 * mb + c][nb] = __builtin_bit_cast(bf16x8, w);
    }
}

// Converts one accumulator tile (D layout: rows 8 g + 4 h + i of M-block mb, values y[16]) of
// a layer's output into the next product's B operands (fp32 and bf16 only).
template <int P, int NKB, int NB>
__device__ inline void tile_to_operands(const float *y, int mb, int nb, typename OpOf<P>::T (&b)[NKB][NB]) {
    if constexpr (P == kBF16) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int s = 0; s < 8; ++s) b[2 * mb + c][nb][s] = (__bf16)y[8 * c + s];
    } else if constexpr (P == kFP8) {
#pragma unroll
        for (int w4 = 0; w4 < 4; ++w4)
            b[mb / 2][nb][4 * (mb % 2) + w4] = pack_fp8x4(y[4 * w4], y[4 * w4 + 1], y[4 * w4 + 2], y[4 * w4 + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) b[16 * mb + j][nb] = y[j];
    }
}

// acc[mb][nb] = sum over the KIN K-blocks of A tile (kb * NMB + mb) x b[kb][nb], with the A
// tiles streamed through a ring loaded kRing steps ahead (tiles are stored K-block major).
template <int P, int NMB, int NB, int KIN, int NKB>
__device__ __attribute__((always_inline)) inline void mfma_tiles(const uint8_t *src, int64_t t0,
                                                                 const typename OpOf<P>::T (&b)[NKB][NB],
                                                                 f32x16 (&acc)[NMB][NB], int lane) {
    using Op = typename OpOf<P>::T;
    constexpr int NSTEP = KIN * NMB;
    constexpr int kRing = P == kFP32 ? 8 : (P == kFP8 ? 2 : 4);   // fp8 tiles are 8 registers each
    Op ring[kRing];
#pragma unroll
    for (int i = 0; i < kRing; ++i) ring[i] = load_a<P>(src, t0 + (i < NSTEP ? i : 0), lane);
#pragma unroll
    for (int step = 0; step < NSTEP; ++step) {
        const int kb = step / NMB, mb = step % NMB;
        const Op a = ring[step % kRing];
        if (step + kRing < NSTEP) ring[step % kRing] = load_a<P>(src, t0 + step + kRing, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma<P>(a, b[kb][nb], kb == 0 ? f32x16{} : acc[mb][nb]);
    }
}

}  // namespace ddf
