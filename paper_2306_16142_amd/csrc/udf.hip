// Unsigned distance field from the directional one (Sec. III-A, Eq. 5): UDF(x) = min over a
// direction set of phi(x, theta), where phi is the network's distance and is infinite where
// the network reports a miss (logit <= 0).
//
// Stages, per chunk of points (as many as the caller's workspace holds):
//   angles   the direction set's (theta, phi) once per call (the shared device definition of
//            Eq. 1 read backwards, bit-identical to ddf_assemble_rays)
//   grid     one thread per (point, direction) query: the network input (x, theta, phi),
//            point-major
//   network  ddf_forward over the chunk's queries (every shape and precision it supports)
//   min      one wave per point: each lane scans a strided share of the directions in
//            ascending order, then a wave reduction keeps the smallest distance and, among
//            equal ones, the lowest direction index
// For networks whose weights fit in LDS the grid, the network and the minimum are one kernel
// (the forward kernel's UDF form: each 32-query block reduces its points' hits to 64-bit keys
// and meets the other blocks in an atomic minimum), then the keys are decoded; the answers
// are the same, since the minimum and its tie rule do not depend on the order.
#include <climits>
#include <cmath>

#include "common.hpp"
#include "rays_device.hpp"

namespace ddf {

bool udf_fused_ok(const ddf_net *net, int64_t np, int64_t nd);
ddf_status udf_fused_launch(const ddf_net *net, const float *points, int64_t np, const float *ang, int64_t nd,
                            unsigned long long *keys, hipStream_t s);

namespace {

constexpr int64_t kUdfMaxQueries = (int64_t)1 << 24;   // queries per chunk the size query plans for
constexpr int kUdfWaves = 4;                              // points per min-reduction block

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__global__ void udf_angles_kernel(const float *__restrict__ dirs, int64_t nd, float *__restrict__ ang) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nd) return;
    float theta, phi;
    dir_angles(dirs[j], dirs[nd + j], dirs[2 * nd + j], theta, phi);
    ang[j] = theta;
    ang[nd + j] = phi;
}

// Query q of the chunk (points p0 .. p0 + nq / nd - 1): point p0 + q / nd, direction q % nd;
// rays [5][nq].
__global__ void udf_grid_kernel(const float *__restrict__ points, int64_t np, int64_t p0, const float *__restrict__ ang,
                                int64_t nd, int64_t nq, float *__restrict__ rays) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const int64_t p = p0 + q / nd, j = q % nd;
#pragma unroll
    for (int c = 0; c < 3; ++c) rays[c * nq + q] = points[c * np + p];
    rays[3 * nq + q] = ang[j];
    rays[4 * nq + q] = ang[nd + j];
}

// Point k of the chunk: min over its nd queries (a NaN distance counts as a miss).
__global__ __launch_bounds__(kUdfWaves * 64) void udf_min_kernel(const float *__restrict__ logit,
                                                                 const float *__restrict__ dist, int64_t nd,
                                                                 int64_t npc, float *__restrict__ udf_out,
                                                                 int32_t *__restrict__ arg_out) {
    const int64_t k = (int64_t)blockIdx.x * kUdfWaves + (threadIdx.x >> 6);
    if (k >= npc) return;
    const int lane = threadIdx.x & 63;
    float best = INFINITY;
    int bi = INT_MAX;
    for (int64_t j = lane; j < nd; j += 64) {
        const int64_t q = k * nd + j;
        const float dd = dist[q];
        if (logit[q] > 0.f && dd < best) {
            best = dd;
            bi = (int)j;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob < best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    if (lane == 0) {
        udf_out[k] = best;
        if (arg_out) arg_out[k] = best < INFINITY ? bi : -1;
    }
}

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

__global__ void udf_keys_init_kernel(unsigned long long *__restrict__ keys, int64_t np) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) keys[i] = ~0ull;
}

// Key = order-preserving bits of the distance (high word), direction index (low word);
// ~0 = every direction missed.
__global__ void udf_keys_decode_kernel(const unsigned long long *__restrict__ keys, int64_t np,
                                       float *__restrict__ udf_out, int32_t *__restrict__ arg_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const unsigned long long k = keys[i];
    const uint32_t ord = (uint32_t)(k >> 32);
    const uint32_t u = (ord & 0x80000000u) ? (ord & 0x7fffffffu) : ~ord;
    udf_out[i] = k == ~0ull ? INFINITY : __uint_as_float(u);
    if (arg_out) arg_out[i] = k == ~0ull ? -1 : (int32_t)(uint32_t)k;
}

// Workspace for chunks of `chunk` points: angles [2][nd] | rays [5][chunk nd] | logit | dist,
// each 256-byte aligned (the three alignments of the per-query arrays are the 768 bytes).
size_t udf_fixed_bytes(int64_t nd) { return align256(8 * nd) + 3 * 256; }
size_t udf_bytes(int64_t chunk, int64_t nd) { return udf_fixed_bytes(nd) + (size_t)28 * chunk * nd; }
// The fused form: angles [2][nd] | keys [np].
size_t udf_fused_bytes(int64_t np, int64_t nd) { return align256(8 * nd) + align256(8 * np); }

}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_udf_workspace_size(int64_t n_points, int64_t n_dirs, size_t *bytes) {
    using namespace ddf;
    DDF_REQUIRE(n_points >= 0 && n_dirs >= 0 && bytes, DDF_ERR_INVALID_ARG, "ddf_udf_workspace_size: bad argument");
    DDF_REQUIRE(n_dirs < ((int64_t)1 << 31), DDF_ERR_UNSUPPORTED, "ddf_udf_workspace_size: too many directions");
    if (n_points == 0 || n_dirs == 0) {
        *bytes = 0;
        return DDF_OK;
    }
    const int64_t chunk = std::min<int64_t>(n_points, std::max<int64_t>(1, kUdfMaxQueries / n_dirs));
    *bytes = std::max(udf_bytes(chunk, n_dirs), udf_fused_bytes(n_points, n_dirs));
    return DDF_OK;
}

extern "C" ddf_status ddf_udf(const ddf_net *net, const float *points, int64_t n_points, const float *dirs,
                              int64_t n_dirs, float *udf_out, int32_t *arg_out, void *ws, size_t ws_bytes,
                              ddf_stream stream) {
    using namespace ddf;
    DDF_REQUIRE(net && net->packed, DDF_ERR_INVALID_ARG, "ddf_udf: NULL network");
    if (ddf_status st = ddf_forward(net, nullptr, 0, nullptr, nullptr, stream)) return st;   // shape check only
    DDF_REQUIRE(n_points >= 0 && n_dirs >= 0, DDF_ERR_INVALID_ARG, "ddf_udf: negative size");
    DDF_REQUIRE(n_dirs < ((int64_t)1 << 31), DDF_ERR_UNSUPPORTED, "ddf_udf: too many directions");
    if (n_points == 0) return DDF_OK;
    DDF_REQUIRE(points && udf_out && (n_dirs == 0 || dirs), DDF_ERR_INVALID_ARG, "ddf_udf: NULL array");
    hipStream_t s = as_stream(stream);
    if (n_dirs == 0) {   // the minimum over no direction: +inf, argument -1
        hipLaunchKernelGGL(udf_min_kernel, dim3(blocks_for(n_points, kUdfWaves)), dim3(kUdfWaves * 64), 0, s,
                           (const float *)nullptr, (const float *)nullptr, (int64_t)0, n_points, udf_out, arg_out);
        return launch_status("ddf_udf");
    }
    if (udf_fused_ok(net, n_points, n_dirs) && ws && ws_bytes >= udf_fused_bytes(n_points, n_dirs)) {
        float *ang = (float *)ws;
        auto *keys = (unsigned long long *)((uint8_t *)ws + align256(8 * n_dirs));
        hipLaunchKernelGGL(udf_keys_init_kernel, dim3(blocks_for(n_points, 256)), dim3(256), 0, s, keys, n_points);
        hipLaunchKernelGGL(udf_angles_kernel, dim3(blocks_for(n_dirs, 256)), dim3(256), 0, s, dirs, n_dirs, ang);
        if (ddf_status st = udf_fused_launch(net, points, n_points, ang, n_dirs, keys, s)) return st;
        hipLaunchKernelGGL(udf_keys_decode_kernel, dim3(blocks_for(n_points, 256)), dim3(256), 0, s, keys, n_points,
                           udf_out, arg_out);
        return launch_status("ddf_udf");
    }
    const size_t fixed = udf_fixed_bytes(n_dirs);
    const size_t per_point = (size_t)28 * n_dirs;
    DDF_REQUIRE(ws && ws_bytes >= fixed + per_point, DDF_ERR_WORKSPACE,
                "ddf_udf: workspace of %zu bytes, need at least %zu (ddf_udf_workspace_size)", ws_bytes,
                fixed + per_point);
    const int64_t chunk = std::min<int64_t>(n_points, (int64_t)((ws_bytes - fixed) / per_point));
    const int64_t cq = chunk * n_dirs;
    uint8_t *base = (uint8_t *)ws;
    float *ang = (float *)base;
    float *rays = (float *)(base + align256(8 * n_dirs));
    float *logit = (float *)((uint8_t *)rays + align256(20 * cq));
    float *dist = (float *)((uint8_t *)logit + align256(4 * cq));
    hipLaunchKernelGGL(udf_angles_kernel, dim3(blocks_for(n_dirs, 256)), dim3(256), 0, s, dirs, n_dirs, ang);
    for (int64_t p0 = 0; p0 < n_points; p0 += chunk) {
        const int64_t npc = std::min<int64_t>(chunk, n_points - p0), nq = npc * n_dirs;
        hipLaunchKernelGGL(udf_grid_kernel, dim3(blocks_for(nq, 256)), dim3(256), 0, s, points, n_points, p0, ang,
                           n_dirs, nq, rays);
        if (ddf_status st = ddf_forward(net, rays, nq, logit, dist, stream)) return st;
        hipLaunchKernelGGL(udf_min_kernel, dim3(blocks_for(npc, kUdfWaves)), dim3(kUdfWaves * 64), 0, s, logit, dist,
                           n_dirs, npc, udf_out + p0, arg_out ? arg_out + p0 : nullptr);
    }
    return launch_status("ddf_udf");
}

// ------------------------------------------------------------------------------ no allocation
// ddf_udf for callers that cannot allocate (code under HIP graph capture, serving loops): its
// scratch -- the direction angles, the fused form's 64-bit keys, or the unfused form's chunks of
// queries -- lives in one file-scope device array per GPU.  Host code never uses the array's
// name as an address: its device address comes from hipGetSymbolAddress, once per device, with
// that device current.
#include <mutex>

namespace ddf {
namespace {

constexpr size_t kUdfScratchBytes = (size_t)8 << 20;   // 8 MiB per GPU, held until the process ends
constexpr int64_t kUdfScratchMaxDirs = 65536;          // one point's queries always fit (2.4 MB)
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kUdfScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (NULL and an error message on failure).
void *udf_scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("ddf_udf_noalloc: no current HIP device (or device index >= %d)", kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("ddf_udf_noalloc: hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_udf_noalloc(const ddf_net *net, const float *points, int64_t n_points, const float *dirs,
                                      int64_t n_dirs, float *udf_out, int32_t *arg_out, ddf_stream stream) {
    using namespace ddf;
    DDF_REQUIRE(n_dirs >= 0 && n_dirs <= kUdfScratchMaxDirs, DDF_ERR_UNSUPPORTED,
                "ddf_udf_noalloc: %lld directions; at most %lld fit the fixed scratch (use ddf_udf with a workspace)",
                (long long)n_dirs, (long long)kUdfScratchMaxDirs);
    void *ws = udf_scratch_ptr();
    if (!ws) return DDF_ERR_HIP;
    return ddf_udf(net, points, n_points, dirs, n_dirs, udf_out, arg_out, ws, kUdfScratchBytes, stream);
}
