// Informative training-data sampler (Sec. V-B, Eqs. 8-12, Fig. 2): points on the faces of
// the mesh (Eq. 8), directions per face (Eq. 9), rejection of rays that meet the mesh again,
// marching samples that look back at the face point (Eq. 10) and infinite samples that look
// on along the ray or to its polar sides (Eqs. 11-12).
//
// Every ray test is the brute-force labeller (label_queue) over all triangles; the rest is
// data movement, so the stages are short kernels over structure-of-arrays buffers in the
// caller's workspace:
//   pairs       one thread per (face point, direction) pair: the origin, direction, angles
//               and exit distance from the domain cube
//   labeller    the pair rays, t_min = eps (the offset that steps over the own face)
//   scan        kept flags -> positions (deterministic: block sums, one scan of the block
//               sums, block-local scans), then the kept pair list
//   perp        one thread per (kept pair, marching step): the line through the marching
//               point along the polar perpendicular
//   labeller    both rays of each line in one test per triangle (line form of the labeller),
//               count read from the device
//   scan        samples per (kept pair, step): 2 + free perpendiculars -> output positions
//   emit        one thread per (kept pair, step): its 2-4 samples at their positions
// Counts stay on the device, so the call never synchronises the host.
#include <cmath>

#include "common.hpp"

namespace ddf {

ddf_status label_queue(const float *orig, const float *dir, int64_t stride, const int *idx, const int *count_dev,
                       const float *tris, int64_t m, float t_min, float t_max, float *t_out, int32_t *tri_out,
                       hipStream_t s);
ddf_status line_queue(const float *orig, const float *dir, int64_t stride, const int *count_dev, const float *tris,
                      int64_t m, int32_t *side_out, hipStream_t s);

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kHalfPi = 1.57079632679489661923f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;                              // per thread
constexpr int kScanBlock = kScanThreads * kScanItems;      // items per block
constexpr int kTopThreads = 1024;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace carve-up for P pairs and s_p steps (U = P * s_p units = perpendicular lines, each
// with a + and a - side).
struct DsWs {
    float *o, *d, *t_exit, *th0, *th1, *t_fwd;
    int32_t *tri_fwd;
    int *cnt, *pos, *acc_idx, *bsum, *counts;   // counts: [0] kept, [1] units, [2] perp rays, [3] samples
    float *po, *pd;
    int32_t *ptri;                              // [2U]: a hit triangle of each side, -1 = none
    size_t bytes;
};

DsWs carve(int64_t P, int64_t s_p, uint8_t *base) {
    const int64_t U = P * s_p, R = 2 * U;
    const int64_t nmax = U > P ? U : P;
    const int64_t nblk = (nmax + kScanBlock - 1) / kScanBlock;
    DsWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        uint8_t *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    w.o = (float *)take(3 * P * 4);
    w.d = (float *)take(3 * P * 4);
    w.t_exit = (float *)take(P * 4);
    w.th0 = (float *)take(P * 4);
    w.th1 = (float *)take(P * 4);
    w.t_fwd = (float *)take(P * 4);
    w.tri_fwd = (int32_t *)take(P * 4);
    w.cnt = (int *)take(nmax * 4);
    w.pos = (int *)take(nmax * 4);
    w.acc_idx = (int *)take(P * 4);
    w.bsum = (int *)take((nblk + 1) * 4);
    w.counts = (int *)take(4 * 4);
    w.po = (float *)take(3 * U * 4);
    w.pd = (float *)take(3 * U * 4);
    w.ptri = (int32_t *)take(R * 4);
    w.bytes = off;
    return w;
}

// Pair i = (face - face_first) * s_fc * s_dr + point * s_dr + direction.
__global__ void ds_pair_kernel(const float *__restrict__ tris, int64_t m, const float *__restrict__ face_uv,
                               const float *__restrict__ dir_uv, int s_fc, int s_dr, int64_t face_first, int64_t P,
                               float *__restrict__ o, float *__restrict__ d, float *__restrict__ t_exit,
                               float *__restrict__ th0_out, float *__restrict__ th1_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int64_t per_face = (int64_t)s_fc * s_dr;
    const int64_t f = face_first + i / per_face;
    const int64_t pc = f * s_fc + (i / s_dr) % s_fc;   // column of the point's uniforms
    const int64_t dc = f * s_dr + i % s_dr;            // column of the direction's uniforms
    // Eq. 8 with the fold of (a, b) outside the face; the test is exact (the float32 sum and
    // its rounding error, Knuth's two-sum), so a sum that float32 rounds to 1 still folds
    float a = face_uv[pc], b = face_uv[m * s_fc + pc];
    const float ab = a + b, bb = ab - a, ab_err = (a - (ab - bb)) + (b - bb);
    if (ab > 1.f || (ab == 1.f && ab_err > 0.f)) {
        a = 1.f - a;
        b = 1.f - b;
    }
    const float w0 = 1.f - a - b;
    float p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = w0 * tris[c * m + f] + a * tris[(3 + c) * m + f] + b * tris[(6 + c) * m + f];
    // Eq. 9: polar angle a pi, azimuth 2 b pi; Eq. 1 for the direction
    const float th0 = dir_uv[dc] * kPi, th1 = dir_uv[m * s_dr + dc] * kTwoPi;
    float s0, c0, s1, c1;
    sincosf(th0, &s0, &c0);
    sincosf(th1, &s1, &c1);
    const float dv[3] = {s0 * c1, s0 * s1, c0};
    // exit from the domain cube [-1, 1]^3; a point outside the cube gives 0 (the pair is dropped)
    float te = INFINITY;
    bool inside = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        inside &= fabsf(p[c]) < 1.f;
        if (dv[c] > 0.f) te = fminf(te, (1.f - p[c]) / dv[c]);
        else if (dv[c] < 0.f) te = fminf(te, (-1.f - p[c]) / dv[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o[c * P + i] = p[c];
        d[c * P + i] = dv[c];
    }
    t_exit[i] = inside ? te : 0.f;
    th0_out[i] = th0;
    th1_out[i] = th1;
}

// A pair is kept when its ray meets no triangle beyond eps and starts inside the cube.
__global__ void ds_keep_kernel(const int32_t *__restrict__ tri_fwd, const float *__restrict__ t_exit, int64_t P,
                               int *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) cnt[i] = (tri_fwd[i] < 0 && t_exit[i] > 0.f) ? 1 : 0;
}

__device__ inline int64_t active_count(int64_t n_max, const int *n_dev) {
    return n_dev ? min<int64_t>(*n_dev, n_max) : n_max;
}

// Inclusive scan of one value per thread over the block (wave shuffles, then the wave totals).
__device__ inline int block_inclusive_scan(int v, int *s_wave) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off);
        if (lane >= off) v += u;
    }
    if (lane == 63) s_wave[wave] = v;
    __syncthreads();
    int carry = 0;
    for (int w = 0; w < wave; ++w) carry += s_wave[w];
    __syncthreads();
    return v + carry;
}

// Scan stage 1: the sum of each block of kScanBlock items.
__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(const int *__restrict__ cnt, int64_t n_max,
                                                                 const int *__restrict__ n_dev, int *__restrict__ bsum) {
    __shared__ int s_wave[kScanThreads / 64];
    const int64_t n = active_count(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    if (base >= n) return;
    int v = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t idx = base + (int64_t)threadIdx.x * kScanItems + j;
        v += idx < n ? cnt[idx] : 0;
    }
    const int incl = block_inclusive_scan(v, s_wave);
    if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = incl;
}

// Scan stage 2 (one workgroup): block sums -> exclusive block offsets, in chunks with a
// running carry.  counts[slot] = total; counts[slot + 1 + j] = total * mul[j] when mul[j] > 0;
// total64 (if given) receives the total too.
__global__ __launch_bounds__(kTopThreads) void scan_top_kernel(int *__restrict__ bsum, int64_t n_max,
                                                               const int *__restrict__ n_dev, int *__restrict__ counts,
                                                               int slot, int mul1, int mul2,
                                                               int64_t *__restrict__ total64) {
    __shared__ int s_wave[kTopThreads / 64];
    __shared__ int s_chunk;
    const int64_t n = active_count(n_max, n_dev);
    const int64_t nblk = (n + kScanBlock - 1) / kScanBlock;
    int carry = 0;
    for (int64_t c0 = 0; c0 < nblk; c0 += kTopThreads) {
        const int64_t b = c0 + threadIdx.x;
        const int v = b < nblk ? bsum[b] : 0;
        const int incl = block_inclusive_scan(v, s_wave);
        if (b < nblk) bsum[b] = carry + incl - v;
        if (threadIdx.x == kTopThreads - 1) s_chunk = incl;   // the chunk's total
        __syncthreads();
        carry += s_chunk;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        counts[slot] = carry;
        if (mul1 > 0) counts[slot + 1] = carry * mul1;
        if (mul2 > 0) counts[slot + 2] = carry * mul2;
        if (total64) *total64 = carry;
    }
}

// Scan stage 3: exclusive positions = block offset + block-local exclusive scan.
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int *__restrict__ cnt, int64_t n_max,
                                                                  const int *__restrict__ n_dev,
                                                                  const int *__restrict__ bsum, int *__restrict__ pos) {
    __shared__ int s_wave[kScanThreads / 64];
    const int64_t n = active_count(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    if (base >= n) return;
    int v[kScanItems], sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t idx = base + (int64_t)threadIdx.x * kScanItems + j;
        v[j] = idx < n ? cnt[idx] : 0;
        sum += v[j];
    }
    int run = block_inclusive_scan(sum, s_wave) - sum + bsum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t idx = base + (int64_t)threadIdx.x * kScanItems + j;
        if (idx < n) pos[idx] = run;
        run += v[j];
    }
}

// Deterministic exclusive scan of cnt[0 .. n) (n = *n_dev if given, else n_max) into pos.
void scan(const int *cnt, int64_t n_max, const int *n_dev, int *pos, int *bsum, int *counts, int slot, int mul1,
          int mul2, int64_t *total64, hipStream_t s) {
    const int64_t nblk = (n_max + kScanBlock - 1) / kScanBlock;
    if (nblk > 0)
        hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, cnt, n_max, n_dev, bsum);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kTopThreads), 0, s, bsum, n_max, n_dev, counts, slot, mul1, mul2,
                       total64);
    if (nblk > 0)
        hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, cnt, n_max, n_dev, bsum,
                           pos);
}

__global__ void ds_compact_kernel(const int *__restrict__ cnt, const int *__restrict__ pos, int64_t P,
                                  int *__restrict__ acc_idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P && cnt[i]) acc_idx[pos[i]] = (int)i;
}

// Marching point k (1..s_p) of kept pair i: q = o + (t_exit k / s_p) d.
__device__ inline void march_point(const float *__restrict__ o, const float *__restrict__ d, float te, int64_t P,
                                   int64_t i, int k, int s_p, float (&q)[3], float &tk) {
    tk = te * (float)k / (float)s_p;
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c] = o[c * P + i] + tk * d[c * P + i];
}

// Unit u = kept slot * s_p + (k - 1): its point and the line along polar angle + pi/2 (its
// - side is the ray at - pi/2).
__global__ void ds_perp_kernel(const int *__restrict__ acc_idx, const int *__restrict__ counts, int s_p, int64_t P,
                               const float *__restrict__ o, const float *__restrict__ d,
                               const float *__restrict__ t_exit, const float *__restrict__ th0,
                               const float *__restrict__ th1, int64_t U, float *__restrict__ po,
                               float *__restrict__ pd) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= counts[1]) return;
    const int64_t i = acc_idx[u / s_p];
    const int k = (int)(u % s_p) + 1;
    float q[3], tk;
    march_point(o, d, t_exit[i], P, i, k, s_p, q, tk);
    float s0, c0, s1, c1;
    sincosf(th0[i], &s0, &c0);
    sincosf(th1[i], &s1, &c1);
    const float dp[3] = {c0 * c1, c0 * s1, -s0};   // d(theta0 + pi/2, theta1)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        po[c * U + u] = q[c];
        pd[c * U + u] = dp[c];
    }
}

__global__ void ds_unit_count_kernel(const int32_t *__restrict__ ptri, const int *__restrict__ counts,
                                     int *__restrict__ cnt) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < counts[1]) cnt[u] = 2 + (ptri[2 * u] < 0 ? 1 : 0) + (ptri[2 * u + 1] < 0 ? 1 : 0);
}

__device__ inline float wrap_2pi(float x) { return x >= kTwoPi ? x - kTwoPi : x; }

// Writes the samples of unit u (kinds: back along -theta with label t_k, on along theta,
// polar +pi/2, polar -pi/2; the last two only where that ray met nothing) at pos[u] onwards.
__global__ void ds_emit_kernel(const int *__restrict__ acc_idx, const int *__restrict__ counts, int s_p, int64_t P,
                               const float *__restrict__ o, const float *__restrict__ d,
                               const float *__restrict__ t_exit, const float *__restrict__ th0s,
                               const float *__restrict__ th1s, const int32_t *__restrict__ ptri,
                               const int *__restrict__ pos, int64_t cap, float *__restrict__ rays_out,
                               float *__restrict__ t_out, int32_t *__restrict__ pair_out) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= counts[1]) return;
    const int64_t i = acc_idx[u / s_p];
    const int k = (int)(u % s_p) + 1;
    float q[3], tk;
    march_point(o, d, t_exit[i], P, i, k, s_p, q, tk);
    const float th0 = th0s[i], th1 = wrap_2pi(th1s[i]);
    const float th1_opp = wrap_2pi(th1 + kPi);
    int64_t at = pos[u];
    auto put = [&](float theta, float phi, float t) {
        if (at < cap) {
#pragma unroll
            for (int c = 0; c < 3; ++c) rays_out[c * cap + at] = q[c];
            rays_out[3 * cap + at] = theta;
            rays_out[4 * cap + at] = phi;
            t_out[at] = t;
            if (pair_out) pair_out[at] = (int32_t)i;
        }
        ++at;
    };
    put(kPi - th0, th1_opp, tk);   // looking back at the face point (Eq. 10)
    put(th0, th1, INFINITY);       // looking on along the kept ray (Eq. 11)
    if (ptri[2 * u] < 0) {         // polar + pi/2 (Eq. 12), folded back over the pole
        const float t = th0 + kHalfPi;
        if (t > kPi) put(kTwoPi - t, th1_opp, INFINITY);
        else put(t, th1, INFINITY);
    }
    if (ptri[2 * u + 1] < 0) {     // polar - pi/2
        const float t = th0 - kHalfPi;
        if (t < 0.f) put(-t, th1_opp, INFINITY);
        else put(t, th1, INFINITY);
    }
}

__global__ void ds_zero_count_kernel(int64_t *count) { *count = 0; }

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

ddf_status check_params(const ddf_dataset_params *p, int64_t *P_out) {
    DDF_REQUIRE(p, DDF_ERR_INVALID_ARG, "ddf dataset: NULL params");
    DDF_REQUIRE(p->s_fc >= 1 && p->s_dr >= 1 && p->s_p >= 1, DDF_ERR_INVALID_ARG,
                "ddf dataset: s_fc, s_dr and s_p must be >= 1 (got %d, %d, %d)", p->s_fc, p->s_dr, p->s_p);
    DDF_REQUIRE(std::isfinite(p->eps) && p->eps >= 0.f, DDF_ERR_INVALID_ARG, "ddf dataset: eps must be finite and >= 0");
    DDF_REQUIRE(p->face_first >= 0 && p->n_faces >= 0, DDF_ERR_INVALID_ARG, "ddf dataset: negative face range");
    const int64_t P = p->n_faces * p->s_fc * p->s_dr;
    DDF_REQUIRE(p->n_faces < ((int64_t)1 << 31) && P / p->s_fc / p->s_dr == p->n_faces &&
                    P * p->s_p < ((int64_t)1 << 29),
                DDF_ERR_UNSUPPORTED, "ddf dataset: n_faces * s_fc * s_dr * s_p must stay below 2^29");
    *P_out = P;
    return DDF_OK;
}

}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_dataset_workspace_size(const ddf_dataset_params *p, size_t *bytes) {
    using namespace ddf;
    int64_t P = 0;
    const ddf_status st = check_params(p, &P);
    if (st != DDF_OK) return st;
    DDF_REQUIRE(bytes, DDF_ERR_INVALID_ARG, "ddf_dataset_workspace_size: NULL bytes");
    *bytes = carve(P, p->s_p, nullptr).bytes;
    return DDF_OK;
}

extern "C" ddf_status ddf_sample_dataset(const float *tris, int64_t m, const ddf_dataset_params *p,
                                         const float *face_uv, const float *dir_uv, float *rays_out, float *t_out,
                                         int32_t *pair_out, int64_t cap, int64_t *count_out, void *ws,
                                         size_t ws_bytes, ddf_stream stream) {
    using namespace ddf;
    int64_t P = 0;
    const ddf_status st = check_params(p, &P);
    if (st != DDF_OK) return st;
    DDF_REQUIRE(m >= 0 && m < ((int64_t)1 << 31), DDF_ERR_INVALID_ARG, "ddf_sample_dataset: bad triangle count");
    DDF_REQUIRE(p->face_first + p->n_faces <= m, DDF_ERR_INVALID_ARG,
                "ddf_sample_dataset: faces %lld..%lld beyond the %lld triangles", (long long)p->face_first,
                (long long)(p->face_first + p->n_faces), (long long)m);
    DDF_REQUIRE(cap >= 0, DDF_ERR_INVALID_ARG, "ddf_sample_dataset: negative capacity");
    DDF_REQUIRE(count_out, DDF_ERR_INVALID_ARG, "ddf_sample_dataset: NULL count_out");
    DDF_REQUIRE(cap == 0 || (rays_out && t_out), DDF_ERR_INVALID_ARG, "ddf_sample_dataset: NULL output arrays");
    hipStream_t s = as_stream(stream);
    if (P == 0) {
        hipLaunchKernelGGL(ds_zero_count_kernel, dim3(1), dim3(1), 0, s, count_out);
        return launch_status("ddf_sample_dataset");
    }
    DDF_REQUIRE(tris && face_uv && dir_uv, DDF_ERR_INVALID_ARG, "ddf_sample_dataset: NULL triangles or uniforms");
    const DsWs need = carve(P, p->s_p, nullptr);
    DDF_REQUIRE(ws && ws_bytes >= need.bytes, DDF_ERR_WORKSPACE,
                "ddf_sample_dataset: workspace of %zu bytes, need %zu (ddf_dataset_workspace_size)", ws_bytes,
                need.bytes);
    const DsWs w = carve(P, p->s_p, (uint8_t *)ws);
    const int s_p = p->s_p;
    const int64_t U = P * s_p, R = 2 * U;
    hipLaunchKernelGGL(ds_pair_kernel, dim3(blocks_for(P, 256)), dim3(256), 0, s, tris, m, face_uv, dir_uv, p->s_fc,
                       p->s_dr, p->face_first, P, w.o, w.d, w.t_exit, w.th0, w.th1);
    ddf_status r = label_queue(w.o, w.d, P, nullptr, nullptr, tris, m, p->eps, INFINITY, w.t_fwd, w.tri_fwd, s);
    if (r != DDF_OK) return r;
    hipLaunchKernelGGL(ds_keep_kernel, dim3(blocks_for(P, 256)), dim3(256), 0, s, w.tri_fwd, w.t_exit, P, w.cnt);
    // counts[0] = kept pairs, counts[1] = kept * s_p units, counts[2] = 2 * units perpendicular rays
    scan(w.cnt, P, nullptr, w.pos, w.bsum, w.counts, 0, s_p, 2 * s_p, nullptr, s);
    hipLaunchKernelGGL(ds_compact_kernel, dim3(blocks_for(P, 256)), dim3(256), 0, s, w.cnt, w.pos, P, w.acc_idx);
    hipLaunchKernelGGL(ds_perp_kernel, dim3(blocks_for(U, 256)), dim3(256), 0, s, w.acc_idx, w.counts, s_p, P, w.o,
                       w.d, w.t_exit, w.th0, w.th1, U, w.po, w.pd);
    r = line_queue(w.po, w.pd, U, w.counts + 1, tris, m, w.ptri, s);
    if (r != DDF_OK) return r;
    hipLaunchKernelGGL(ds_unit_count_kernel, dim3(blocks_for(U, 256)), dim3(256), 0, s, w.ptri, w.counts, w.cnt);
    // counts[3] = samples
    scan(w.cnt, U, w.counts + 1, w.pos, w.bsum, w.counts, 3, 0, 0, count_out, s);
    hipLaunchKernelGGL(ds_emit_kernel, dim3(blocks_for(U, 256)), dim3(256), 0, s, w.acc_idx, w.counts, s_p, P, w.o,
                       w.d, w.t_exit, w.th0, w.th1, w.ptri, w.pos, cap, rays_out, t_out, pair_out);
    return launch_status("ddf_sample_dataset");
}
