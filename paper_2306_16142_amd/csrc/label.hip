// Brute-force nearest ray/triangle hit: the linear search over all triangles that the
// paper's field replaces (Sec. I) and the ray shooting that produces its labels
// (Sec. VI-B), with the crossing count of the odd-even inside rule (Sec. V-B).
//
// One lane per ray, 256 rays per workgroup; triangles are staged through LDS in
// tiles of 256 (corner v0, float32 edges e1 = v1 - v0, e2 = v2 - v0, the longest edge
// and |v0|), so every lane tests the same triangle at the same time (broadcast reads).
//
// Each test is the two-sided Moller-Trumbore form in float32 with its decisions taken
// on unnormalised quantities (det, u*det, v*det, t*det) against a forward error bound
// B = 32 eps (|o| + |v0| + L) L |d|: a test is a sure miss or a sure hit when every
// comparison clears its bound, otherwise it is re-evaluated in float64 from the same
// float32 inputs.  The winner's distance is always recomputed in float64, so the
// reported t does not suffer float32 cancellation on small or grazing triangles.
#include <cmath>

#include "common.hpp"

namespace ddf {
namespace {

constexpr int kLabelThreads = 256;
constexpr int kLabelTile = 256;
constexpr float kErr = 32.0f * 5.9604645e-8f;   // 32 unit roundoffs of float32

struct alignas(16) TriLds {
    float v0x, v0y, v0z, L;
    float e1x, e1y, e1z, s;    // s = |v0| + L (the triangle's part of the bound's scale)
    float e2x, e2y, e2z, kL;   // kL = 32 eps L
};

// Float64 Moller-Trumbore from the float32 corners; returns the accepted t or NaN.
__device__ __noinline__ double mt_fp64(const float *__restrict__ tris, int64_t m, int64_t i, double ox,
                                       double oy, double oz, double dx, double dy, double dz, double t_min,
                                       double t_max) {
    const double v0x = tris[0 * m + i], v0y = tris[1 * m + i], v0z = tris[2 * m + i];
    const double e1x = (double)tris[3 * m + i] - v0x, e1y = (double)tris[4 * m + i] - v0y,
                 e1z = (double)tris[5 * m + i] - v0z;
    const double e2x = (double)tris[6 * m + i] - v0x, e2y = (double)tris[7 * m + i] - v0y,
                 e2z = (double)tris[8 * m + i] - v0z;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const double det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0) return NAN;
    const double sx = ox - v0x, sy = oy - v0y, sz = oz - v0z;
    const double u = (sx * px + sy * py + sz * pz) / det;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    const double v = (dx * qx + dy * qy + dz * qz) / det;
    const double t = (e2x * qx + e2y * qy + e2z * qz) / det;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t > t_min && t < t_max) return t;
    return NAN;
}

// Corner v0, edges, longest edge and the bound's scale of triangle i, for the LDS tile.
__device__ inline TriLds stage_triangle(const float *__restrict__ tris, int64_t m, int64_t i) {
    TriLds t;
    t.v0x = tris[i];
    t.v0y = tris[m + i];
    t.v0z = tris[2 * m + i];
    const float v1x = tris[3 * m + i], v1y = tris[4 * m + i], v1z = tris[5 * m + i];
    const float v2x = tris[6 * m + i], v2y = tris[7 * m + i], v2z = tris[8 * m + i];
    t.e1x = v1x - t.v0x;
    t.e1y = v1y - t.v0y;
    t.e1z = v1z - t.v0z;
    t.e2x = v2x - t.v0x;
    t.e2y = v2y - t.v0y;
    t.e2z = v2z - t.v0z;
    const float fx = v2x - v1x, fy = v2y - v1y, fz = v2z - v1z;
    const float l1 = t.e1x * t.e1x + t.e1y * t.e1y + t.e1z * t.e1z;
    const float l2 = t.e2x * t.e2x + t.e2y * t.e2y + t.e2z * t.e2z;
    const float l3 = fx * fx + fy * fy + fz * fz;
    t.L = sqrtf(fmaxf(l1, fmaxf(l2, l3))) * 1.0001f;
    t.s = sqrtf(t.v0x * t.v0x + t.v0y * t.v0y + t.v0z * t.v0z) * 1.0001f + t.L;
    t.kL = kErr * t.L;
    return t;
}

// Output slot q reads ray idx[q] (or q) from [3][stride] arrays; only q < n (or *count_dev)
// are processed.  Blocks past the count exit before touching LDS.
// kTmaxInf: t_max is +inf (labels), so the far bound needs no test.
template <bool kTmaxInf>
__global__ __launch_bounds__(kLabelThreads) void label_kernel(
    const float *__restrict__ orig, const float *__restrict__ dir, int64_t stride, const int *__restrict__ idx,
    const int *__restrict__ count_dev, const float *__restrict__ tris, int64_t m, float t_min, float t_max,
    float *__restrict__ t_out, int32_t *__restrict__ tri_out, uint32_t *__restrict__ cross_out) {
    __shared__ TriLds s_tri[kLabelTile];
    const int64_t n = count_dev ? min<int64_t>(*count_dev, stride) : stride;
    if ((int64_t)blockIdx.x * kLabelThreads >= n) return;
    const int64_t ray = (int64_t)blockIdx.x * kLabelThreads + threadIdx.x;
    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f;
    if (ray < n) {
        const int64_t src = idx ? (int64_t)idx[ray] : ray;
        ox = orig[src];
        oy = orig[stride + src];
        oz = orig[2 * stride + src];
        dx = dir[src];
        dy = dir[stride + src];
        dz = dir[2 * stride + src];
    }
    const bool finite = isfinite(ox) && isfinite(oy) && isfinite(oz) && isfinite(dx) && isfinite(dy) &&
                        isfinite(dz) && (dx != 0.f || dy != 0.f || dz != 0.f);
    const bool active = ray < n && finite;
    const float onorm = sqrtf(ox * ox + oy * oy + oz * oz);
    const float dnorm = sqrtf(dx * dx + dy * dy + dz * dz);
    constexpr bool tmax_inf = kTmaxInf;
    const float abs_tmin = fabsf(t_min), abs_tmax = tmax_inf ? 0.f : fabsf(t_max);

    float best_t = INFINITY;
    int32_t best_i = -1;
    uint32_t cross = 0;

    for (int64_t base = 0; base < m; base += kLabelTile) {
        const int cnt = (int)min<int64_t>(kLabelTile, m - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) s_tri[threadIdx.x] = stage_triangle(tris, m, base + threadIdx.x);
        __syncthreads();
        if (!active) continue;
        for (int k = 0; k < cnt; ++k) {
            const TriLds T = s_tri[k];
            const float px = dy * T.e2z - dz * T.e2y;
            const float py = dz * T.e2x - dx * T.e2z;
            const float pz = dx * T.e2y - dy * T.e2x;
            const float D0 = T.e1x * px + T.e1y * py + T.e1z * pz;
            const float sx = ox - T.v0x, sy = oy - T.v0y, sz = oz - T.v0z;
            const float qx = sy * T.e1z - sz * T.e1y;
            const float qy = sz * T.e1x - sx * T.e1z;
            const float qz = sx * T.e1y - sy * T.e1x;
            // the two-sided test on |det|: flip the signs of all four quantities with det's
            const uint32_t sgn = __float_as_uint(D0) & 0x80000000u;
            const float D = __uint_as_float(__float_as_uint(D0) ^ sgn);
            const float U = __uint_as_float(__float_as_uint(sx * px + sy * py + sz * pz) ^ sgn);
            const float V = __uint_as_float(__float_as_uint(dx * qx + dy * qy + dz * qz) ^ sgn);
            const float Tq = __uint_as_float(__float_as_uint(T.e2x * qx + T.e2y * qy + T.e2z * qz) ^ sgn);
            const float st = (onorm + T.s) * T.kL;   // 32 eps (|o| + |v0| + L) L
            const float B = st * dnorm;
            const float BT = st * T.L;
            // sure miss (no lane of the wave needs more: the common case, one branch per wave)
            const bool small = D <= 2.f * B;
            const float lo = t_min * D, blo = BT + abs_tmin * B;
            const float hi = tmax_inf ? INFINITY : t_max * D, bhi = BT + abs_tmax * B;
            // every comparison as a wave-wide lane mask (scalar ORs, no per-lane branch)
            const uint64_t m_small = __ballot(small);
            const uint64_t ms = __ballot(fabsf(U) > 4.f * B) | __ballot(fabsf(V) > 4.f * B);
            uint64_t mb = __ballot(U < -B) | __ballot(V < -B) | __ballot(U + V > D + 3.f * B) | __ballot(Tq <= lo - blo);
            if constexpr (!kTmaxInf) mb |= __ballot(Tq >= hi + bhi);
            const uint64_t miss_mask = (m_small & ms) | (~m_small & mb);
            if (__builtin_expect((__ballot(1) & ~miss_mask) == 0, 1)) continue;
            const bool miss = (miss_mask >> __lane_id()) & 1u;
            int decision;   // 0 sure miss, 1 sure hit, 2 undecided
            if (miss) {
                decision = 0;
            } else if (small) {
                decision = 2;
            } else {
                const bool hit = U > B && V > B && U + V < D - 3.f * B && Tq > lo + blo && (tmax_inf || Tq < hi - bhi);
                decision = hit ? 1 : 2;
            }
            if (decision == 0) continue;
            float t;
            if (decision == 1) {
                t = Tq / D;
            } else {
                const double t64 = mt_fp64(tris, m, base + k, ox, oy, oz, dx, dy, dz, t_min, t_max);
                if (isnan(t64)) continue;
                t = (float)t64;
            }
            ++cross;
            if (t < best_t) {
                best_t = t;
                best_i = (int32_t)(base + k);
            }
        }
    }
    if (ray >= n) return;
    if (best_i >= 0) {
        // Report the winner's distance from a float64 evaluation of the same test.
        const double t64 = mt_fp64(tris, m, best_i, ox, oy, oz, dx, dy, dz, -INFINITY, INFINITY);
        if (!isnan(t64)) best_t = (float)t64;
    }
    t_out[ray] = best_t;
    tri_out[ray] = best_i;
    if (cross_out) cross_out[ray] = cross;
}

// Any hit on both rays of a line: from `orig` along +dir and along -dir (t > 0 on each side),
// with one Moller-Trumbore test per triangle.  For -dir the float32 quantities are exactly
// those of +dir with det and t*det negated (so u, v and |det| agree and t changes sign), and
// the float64 re-evaluation negates exactly too, so each side's decision equals the one the
// labeller takes for that ray on its own (t_min = 0, t_max = +inf).
// side_out[2 q] and [2 q + 1]: the index of a triangle hit on the + and - side (the first
// met, not the nearest), -1 where that side meets nothing; lines q < *count_dev (or stride)
// read [3][stride] arrays.
__global__ __launch_bounds__(kLabelThreads) void line_kernel(const float *__restrict__ orig,
                                                             const float *__restrict__ dir, int64_t stride,
                                                             const int *__restrict__ count_dev,
                                                             const float *__restrict__ tris, int64_t m,
                                                             int32_t *__restrict__ side_out) {
    __shared__ TriLds s_tri[kLabelTile];
    const int64_t n = count_dev ? min<int64_t>(*count_dev, stride) : stride;
    if ((int64_t)blockIdx.x * kLabelThreads >= n) return;
    const int64_t ray = (int64_t)blockIdx.x * kLabelThreads + threadIdx.x;
    float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f;
    if (ray < n) {
        ox = orig[ray];
        oy = orig[stride + ray];
        oz = orig[2 * stride + ray];
        dx = dir[ray];
        dy = dir[stride + ray];
        dz = dir[2 * stride + ray];
    }
    const bool finite = isfinite(ox) && isfinite(oy) && isfinite(oz) && isfinite(dx) && isfinite(dy) &&
                        isfinite(dz) && (dx != 0.f || dy != 0.f || dz != 0.f);
    const bool active = ray < n && finite;
    const float onorm = sqrtf(ox * ox + oy * oy + oz * oz);
    const float dnorm = sqrtf(dx * dx + dy * dy + dz * dz);
    int32_t hit_p = -1, hit_m = -1;
    for (int64_t base = 0; base < m; base += kLabelTile) {
        const int cnt = (int)min<int64_t>(kLabelTile, m - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) s_tri[threadIdx.x] = stage_triangle(tris, m, base + threadIdx.x);
        __syncthreads();
        if (!active) continue;
        for (int k = 0; k < cnt; ++k) {
            const TriLds T = s_tri[k];
            const float px = dy * T.e2z - dz * T.e2y;
            const float py = dz * T.e2x - dx * T.e2z;
            const float pz = dx * T.e2y - dy * T.e2x;
            const float D0 = T.e1x * px + T.e1y * py + T.e1z * pz;
            const float sx = ox - T.v0x, sy = oy - T.v0y, sz = oz - T.v0z;
            const float qx = sy * T.e1z - sz * T.e1y;
            const float qy = sz * T.e1x - sx * T.e1z;
            const float qz = sx * T.e1y - sy * T.e1x;
            const uint32_t sgn = __float_as_uint(D0) & 0x80000000u;
            const float D = __uint_as_float(__float_as_uint(D0) ^ sgn);
            const float U = __uint_as_float(__float_as_uint(sx * px + sy * py + sz * pz) ^ sgn);
            const float V = __uint_as_float(__float_as_uint(dx * qx + dy * qy + dz * qz) ^ sgn);
            const float Tq = __uint_as_float(__float_as_uint(T.e2x * qx + T.e2y * qy + T.e2z * qz) ^ sgn);
            const float st = (onorm + T.s) * T.kL;
            const float B = st * dnorm;
            const float BT = st * T.L;
            // sure miss of both sides: the line passes outside the triangle (no test on t)
            const bool small = D <= 2.f * B;
            const uint64_t m_small = __ballot(small);
            const uint64_t ms = __ballot(fabsf(U) > 4.f * B) | __ballot(fabsf(V) > 4.f * B);
            const uint64_t mb = __ballot(U < -B) | __ballot(V < -B) | __ballot(U + V > D + 3.f * B);
            const uint64_t miss_mask = (m_small & ms) | (~m_small & mb);
            if (__builtin_expect((__ballot(1) & ~miss_mask) == 0, 1)) continue;
            if ((miss_mask >> __lane_id()) & 1u) continue;
            if (hit_p >= 0 && hit_m >= 0) continue;
            const int32_t idx = (int32_t)(base + k);
            const bool inside = !small && U > B && V > B && U + V < D - 3.f * B;
            if (inside && Tq > BT) {
                if (hit_p < 0) hit_p = idx;
            } else if (inside && Tq < -BT) {
                if (hit_m < 0) hit_m = idx;
            } else {   // undecided: each side in float64 from the same float32 inputs
                if (hit_p < 0 && !isnan(mt_fp64(tris, m, idx, ox, oy, oz, dx, dy, dz, 0.0, INFINITY))) hit_p = idx;
                if (hit_m < 0 && !isnan(mt_fp64(tris, m, idx, ox, oy, oz, -dx, -dy, -dz, 0.0, INFINITY)))
                    hit_m = idx;
            }
        }
    }
    if (ray >= n) return;
    side_out[2 * ray] = hit_p;
    side_out[2 * ray + 1] = hit_m;
}

}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_label_rays(const float *orig, const float *dir, int64_t n, const float *tris, int64_t m,
                                     float t_min, float t_max, float *t_out, int32_t *tri_out, uint32_t *crossings,
                                     ddf_stream stream) {
    using namespace ddf;
    DDF_REQUIRE(n >= 0 && m >= 0, DDF_ERR_INVALID_ARG, "ddf_label_rays: negative size (n=%lld, m=%lld)",
                (long long)n, (long long)m);
    DDF_REQUIRE(!(t_min >= t_max) && !std::isnan(t_min) && !std::isnan(t_max), DDF_ERR_INVALID_ARG,
                "ddf_label_rays: need t_min < t_max");
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(orig && dir && t_out && tri_out, DDF_ERR_INVALID_ARG, "ddf_label_rays: NULL ray or output array");
    DDF_REQUIRE(m == 0 || tris, DDF_ERR_INVALID_ARG, "ddf_label_rays: NULL triangle array");
    DDF_REQUIRE(m < (int64_t)1 << 31, DDF_ERR_UNSUPPORTED, "ddf_label_rays: more than 2^31 triangles");
    const int64_t blocks = (n + kLabelThreads - 1) / kLabelThreads;
    DDF_REQUIRE(blocks < (int64_t)1 << 31, DDF_ERR_UNSUPPORTED, "ddf_label_rays: too many rays");
    hipLaunchKernelGGL(std::isinf(t_max) ? label_kernel<true> : label_kernel<false>, dim3((unsigned)blocks),
                       dim3(kLabelThreads), 0, as_stream(stream), orig, dir,
                       n, (const int *)nullptr, (const int *)nullptr, tris, m, t_min, t_max, t_out, tri_out, crossings);
    return launch_status("ddf_label_rays");
}

namespace ddf {
// Both sides of each line q < *count_dev of [3][stride] arrays (see line_kernel).
ddf_status line_queue(const float *orig, const float *dir, int64_t stride, const int *count_dev, const float *tris,
                      int64_t m, int32_t *side_out, hipStream_t s) {
    const int64_t blocks = (stride + kLabelThreads - 1) / kLabelThreads;
    hipLaunchKernelGGL(line_kernel, dim3((unsigned)blocks), dim3(kLabelThreads), 0, s, orig, dir, stride, count_dev, tris,
                       m, side_out);
    return launch_status("ddf labeller (lines)");
}

// Labeller over a queue: slot q < *count_dev reads ray idx[q] of [3][stride] arrays.
ddf_status label_queue(const float *orig, const float *dir, int64_t stride, const int *idx, const int *count_dev,
                       const float *tris, int64_t m, float t_min, float t_max, float *t_out, int32_t *tri_out,
                       hipStream_t s) {
    const int64_t blocks = (stride + kLabelThreads - 1) / kLabelThreads;
    hipLaunchKernelGGL(std::isinf(t_max) ? label_kernel<true> : label_kernel<false>, dim3((unsigned)blocks),
                       dim3(kLabelThreads), 0, s, orig, dir, stride, idx,
                       count_dev, tris, m, t_min, t_max, t_out, tri_out, (uint32_t *)nullptr);
    return launch_status("ddf labeller (queue)");
}
}  // namespace ddf
