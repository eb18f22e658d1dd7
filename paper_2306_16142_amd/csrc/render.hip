// Wavefront path tracer of Fig. 1 with the network (or the brute-force triangle search)
// answering every nearest-hit query: the "modified path tracer" of Sec. I / Sec. IV.
//
// Paths live in structure-of-arrays state indexed by path id; each bounce works on a
// queue of live path ids: prepare the network inputs (cube entry, angles) -> one
// kernel gives logit, distance and d(distance)/d(origin) for the whole queue (the
// normal of Eq. 3) -> shade: next-event ray towards the light, cosine scatter, Russian
// roulette, compaction of survivors and shadow rays with a wave ballot and one atomic
// per wave -> shadow query -> resolve.  Queue lengths stay on the device: every kernel
// is launched for the chunk's capacity and reads its count, so a whole render is a
// fixed sequence of launches with no host synchronisation.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "rays_device.hpp"
#include "tuning.hpp"
#include "mlp_layout.hpp"
#include "grad_args.hpp"

namespace ddf {


ddf_status forward_dispatch(const ddf_net *net, const float *rays, int64_t n, const int *count_dev, float *logit,
                            float *dist, unsigned int *absmax, hipStream_t s);
ddf_status label_queue(const float *orig, const float *dir, int64_t stride, const int *idx, const int *count_dev,
                       const float *tris, int64_t m, float t_min, float t_max, float *t_out, int32_t *tri_out,
                       hipStream_t s);

namespace {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kBelowTwoPi = 6.28318500518798828125f;
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

// ------------------------------------------------------------------------------ RNG
__device__ inline uint64_t sm_hash(uint64_t x) {
    uint64_t z = x + kGolden;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ inline uint64_t path_key(uint64_t seed, uint64_t pixel, uint64_t sample) {
    return sm_hash(sm_hash(sm_hash(seed) ^ pixel) ^ sample);
}
__device__ inline float uniform01(uint64_t key, uint64_t bounce, uint64_t dim) {
    const uint64_t k = sm_hash(sm_hash(key ^ bounce) ^ dim);
    return (float)(k >> 40) * 5.9604644775390625e-8f;   // 2^-24
}

struct Vec3 {
    float x, y, z;
};
__device__ inline Vec3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ inline Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline Vec3 operator*(float s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline float dot(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline Vec3 cross(Vec3 a, Vec3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline Vec3 normalize(Vec3 a) { return (1.0f / sqrtf(dot(a, a))) * a; }
__device__ inline Vec3 load3(const float *p, int64_t stride, int64_t i) { return {p[i], p[stride + i], p[2 * stride + i]}; }
__device__ inline void store3(float *p, int64_t stride, int64_t i, Vec3 v) {
    p[i] = v.x;
    p[stride + i] = v.y;
    p[2 * stride + i] = v.z;
}

// Slab test against [-1,1]^3: entry offset max(t_in, 0), or NaN when the ray misses the cube.
__device__ inline float cube_entry(Vec3 o, Vec3 d) {
    float lo = -INFINITY, hi = INFINITY;
    const float oc[3] = {o.x, o.y, o.z}, dc[3] = {d.x, d.y, d.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (dc[k] == 0.f) {
            if (oc[k] < -1.f || oc[k] > 1.f) return NAN;
        } else {
            const float inv = 1.0f / dc[k];
            const float t0 = (-1.f - oc[k]) * inv, t1 = (1.f - oc[k]) * inv;
            lo = fmaxf(lo, fminf(t0, t1));
            hi = fminf(hi, fmaxf(t0, t1));
        }
    }
    if (!(lo <= hi) || !(hi > 0.f)) return NAN;
    return fmaxf(lo, 0.f);
}

// Network input of a ray: entry point and (polar, azimuth) of the direction.
__device__ inline void write_query(float *rays5, int64_t stride, int64_t q, Vec3 o, Vec3 d, float t0) {
    const float t = isnan(t0) ? 0.f : t0;
    const Vec3 p = o + t * d;
    float theta, phi;
    dir_angles(d.x, d.y, d.z, theta, phi);
    rays5[q] = p.x;
    rays5[stride + q] = p.y;
    rays5[2 * stride + q] = p.z;
    rays5[3 * stride + q] = theta;
    rays5[4 * stride + q] = phi;
}

// Wave-aggregated append: returns this lane's slot (or -1 when it does not append).
__device__ inline int append(int *counter, bool want) {
    const uint64_t mask = __ballot(want);
    if (mask == 0) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(mask));
    base = __shfl(base, leader);
    const int rank = (int)__popcll(mask & ((1ull << lane) - 1ull));
    return want ? base + rank : -1;
}

// Block-aggregated append to two queues at once: every thread of the block must call it
// (the same number of times).  Waves rank their lanes with ballots, wave leaders take
// offsets from LDS counters, and one thread per block reserves the block's ranges in the
// global counters: two global atomics per block and call instead of two per wave (on the
// same two counters, per-wave atomics serialise).  Slot order inside a queue varies between
// runs; consumers address paths by id, so results do not.
struct Append2 {
    int a, b;   // per-wave offsets (LDS), then the block bases
};

__device__ inline void block_append2(int *ctr_a, bool want_a, int *ctr_b, bool want_b, Append2 *s, int &slot_a,
                                     int &slot_b) {
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        s->a = 0;
        s->b = 0;
    }
    __syncthreads();
    const uint64_t ma = __ballot(want_a), mb = __ballot(want_b);
    const uint64_t below = (1ull << lane) - 1ull;
    int wa = 0, wb = 0;
    if (lane == 0) {
        wa = ma ? atomicAdd(&s->a, (int)__popcll(ma)) : 0;
        wb = mb ? atomicAdd(&s->b, (int)__popcll(mb)) : 0;
    }
    wa = __shfl(wa, 0);
    wb = __shfl(wb, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int ta = s->a, tb = s->b;
        s->a = ta ? atomicAdd(ctr_a, ta) : 0;
        s->b = tb ? atomicAdd(ctr_b, tb) : 0;
    }
    __syncthreads();
    slot_a = want_a ? s->a + wa + (int)__popcll(ma & below) : -1;
    slot_b = want_b ? s->b + wb + (int)__popcll(mb & below) : -1;
    __syncthreads();   // s is reused by the next call
}

// ------------------------------------------------------------------------------ multi-object
struct InstDev {
    float R[9];
    float T[3];
    int net;
    float r2;   // squared radius of a world sphere about T holding the instance's cube (INF: none)
    int pad[2];
};
constexpr int kMaxInstances = 64;
constexpr int kMaxCullBlocks = 8192;   // workgroups of one culling pass
constexpr int kInstChunk = 8;
struct InstChunk {
    InstDev v[kInstChunk];
};

__global__ void inst_table_kernel(InstChunk c, int first, int count, InstDev *dst) {
    const int i = threadIdx.x;
    if (i < count) dst[first + i] = c.v[i];
}

// World ray -> object space of instance `in` (x_obj = R^T (x - T)).
__device__ inline void to_object(const InstDev &in, Vec3 o, Vec3 d, Vec3 &oo, Vec3 &dd) {
    const Vec3 s = o - v3(in.T[0], in.T[1], in.T[2]);
    oo = v3(in.R[0] * s.x + in.R[3] * s.y + in.R[6] * s.z, in.R[1] * s.x + in.R[4] * s.y + in.R[7] * s.z,
            in.R[2] * s.x + in.R[5] * s.y + in.R[8] * s.z);
    dd = v3(in.R[0] * d.x + in.R[3] * d.y + in.R[6] * d.z, in.R[1] * d.x + in.R[4] * d.y + in.R[7] * d.z,
            in.R[2] * d.x + in.R[5] * d.y + in.R[8] * d.z);
}

struct PairBufs {
    int *q, *inst;        // [P]
    float *rays5, *t0;    // [5][P], [P]
    float *logit, *dist;  // [P]
    float *grad;          // [5][P]
    float *ones;          // [P]
};

struct MultiCounts {
    int *inst_count, *inst_cursor, *inst_off;   // [kMaxInstances]
    int *seg_offset, *seg_count;                // [n_nets]
    int *total;                                 // [1]
    int *block_count;                           // [culling block][kMaxInstances]: pass 0's counts
};

struct PathState {
    float *o, *d, *thr, *L;   // [3][C]
    int *pix, *smp;           // [C]
};

struct RenderWs {
    PathState ps;
    int *qa, *qb, *counts;
    // single-network and mesh scenes (after every other buffer): queue position -> query slot
    // (-1: the ray misses the cube [-1, 1]^3 and is not queried), and per bounce its hits
    // [bounces] and the rays of its nearest-hit pass [bounces]
    int *cmap, *xcounts;
    float *rays5, *t0, *logit, *dist, *grad, *ones;
    float *tq;
    int *triq;
    int *sq;
    float *srays, *st0, *stmax, *scontrib, *slogit, *sdist, *st;
    int *stri;
    // multi-object scenes
    PairBufs pb;
    int64_t P;
    unsigned long long *best;
    float *hit_t, *hit_g;
    int *occl;
    InstDev *inst;
    MultiCounts mc;
    size_t bytes;
};

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

RenderWs render_ws(int64_t C, int bounces, int n_inst, void *base) {
    RenderWs w{};
    uint8_t *p = reinterpret_cast<uint8_t *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *q = p ? p + off : nullptr;
        off += a256(bytes);
        return q;
    };
    const size_t f = (size_t)C * 4;
    w.ps.o = (float *)take(3 * f);
    w.ps.d = (float *)take(3 * f);
    w.ps.thr = (float *)take(3 * f);
    w.ps.L = (float *)take(3 * f);
    w.ps.pix = (int *)take(f);
    w.ps.smp = (int *)take(f);
    w.qa = (int *)take(f);
    w.qb = (int *)take(f);
    w.counts = (int *)take((size_t)(2 * bounces + 4) * 4);
    w.rays5 = (float *)take(5 * f);
    w.t0 = (float *)take(f);
    w.logit = (float *)take(f);
    w.dist = (float *)take(f);
    w.grad = (float *)take(5 * f);
    w.ones = (float *)take(f);
    w.tq = (float *)take(f);
    w.triq = (int *)take(f);
    w.sq = (int *)take(f);
    w.srays = (float *)take(6 * f);
    w.st0 = (float *)take(f);
    w.stmax = (float *)take(f);
    w.scontrib = (float *)take(3 * f);
    w.slogit = (float *)take(f);
    w.sdist = (float *)take(f);
    w.st = (float *)take(f);
    w.stri = (int *)take(f);
    if (n_inst > 0) {
        const int64_t P = C * n_inst;
        const size_t pf = (size_t)P * 4;
        w.P = P;
        w.pb.q = (int *)take(pf);
        w.pb.inst = (int *)take(pf);
        w.pb.rays5 = (float *)take(5 * pf);
        w.pb.t0 = (float *)take(pf);
        w.pb.logit = (float *)take(pf);
        w.pb.dist = (float *)take(pf);
        w.pb.grad = (float *)take(5 * pf);
        w.pb.ones = (float *)take(pf);
        w.best = (unsigned long long *)take((size_t)C * 8);
        w.hit_t = (float *)take(f);
        w.hit_g = (float *)take(3 * f);
        w.occl = (int *)take(f);
        w.inst = (InstDev *)take(sizeof(InstDev) * kMaxInstances);
        w.mc.inst_count = (int *)take(4 * kMaxInstances);
        w.mc.inst_cursor = (int *)take(4 * kMaxInstances);
        w.mc.inst_off = (int *)take(4 * kMaxInstances);
        w.mc.seg_offset = (int *)take(4 * 2 * kMaxNets);
        w.mc.seg_count = (int *)take(4 * 2 * kMaxNets);
        w.mc.total = (int *)take(16);
        w.mc.block_count = (int *)take((size_t)kMaxCullBlocks * kMaxInstances * 4);
    }
    if (n_inst == 0) {
        w.cmap = (int *)take(f);
        w.xcounts = (int *)take((size_t)2 * bounces * 4);
    }
    w.bytes = off;
    return w;
}

struct Cam {
    Vec3 eye, f, r, u;
    float th, aspect;
};

Cam make_cam(const ddf_render_params &p) {
    auto norm = [](float a[3]) {
        const float l = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        a[0] /= l;
        a[1] /= l;
        a[2] /= l;
    };
    float f[3] = {p.target[0] - p.eye[0], p.target[1] - p.eye[1], p.target[2] - p.eye[2]};
    norm(f);
    float r[3] = {f[1] * p.up[2] - f[2] * p.up[1], f[2] * p.up[0] - f[0] * p.up[2], f[0] * p.up[1] - f[1] * p.up[0]};
    norm(r);
    float u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    Cam c;
    c.eye = {p.eye[0], p.eye[1], p.eye[2]};
    c.f = {f[0], f[1], f[2]};
    c.r = {r[0], r[1], r[2]};
    c.u = {u[0], u[1], u[2]};
    c.th = (float)std::tan(p.vfov_deg * 3.14159265358979323846 / 360.0);
    c.aspect = (float)p.width / (float)p.height;
    return c;
}

// ------------------------------------------------------------------------------ kernels
__global__ void raygen_kernel(ddf_render_params p, Cam cam, int64_t C, int sample_base, int S, PathState ps, int *queue,
                              int *counts, int ncounts, float *ones, float *depth, float *normal) {
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < ncounts; i += blockDim.x) counts[i] = i == 0 ? (int)C : 0;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < C; id += (int64_t)gridDim.x * blockDim.x) {
        const int pixel = (int)(id / S);
        const int sample = sample_base + (int)(id % S);
        const uint64_t key = path_key(p.seed, (uint64_t)pixel, (uint64_t)sample);
        float jx = 0.5f, jy = 0.5f;
        if (p.spp > 1) {
            jx = uniform01(key, 0, 0);
            jy = uniform01(key, 0, 1);
        }
        const float px = (float)(pixel % p.width), py = (float)(pixel / p.width);
        const float sx = (2.0f * (px + jx) / (float)p.width - 1.0f) * cam.th * cam.aspect;
        const float sy = (1.0f - 2.0f * (py + jy) / (float)p.height) * cam.th;
        const Vec3 d = normalize(cam.f + sx * cam.r + sy * cam.u);
        store3(ps.o, C, id, cam.eye);
        store3(ps.d, C, id, d);
        store3(ps.thr, C, id, v3(1.f, 1.f, 1.f));
        store3(ps.L, C, id, v3(0.f, 0.f, 0.f));
        ps.pix[id] = pixel;
        ps.smp[id] = sample;
        queue[id] = (int)id;
        ones[id] = 1.0f;
        if (sample == 0) {
            if (depth) depth[pixel] = INFINITY;
            if (normal) {
                const int64_t hw = (int64_t)p.width * p.height;
                normal[pixel] = 0.f;
                normal[hw + pixel] = 0.f;
                normal[2 * hw + pixel] = 0.f;
            }
        }
    }
}

// Network scenes: the queue's rays that enter the cube [-1, 1]^3 (where the field is
// defined; a ray that misses it misses the object) become the bounce's network queries,
// compacted; cmap[q] is the query slot of queue position q, or -1.
__global__ void prep_kernel(int64_t C, const int *__restrict__ queue, const int *__restrict__ count, PathState ps,
                            float *__restrict__ rays5, float *__restrict__ t0, int *__restrict__ cmap,
                            int *__restrict__ query_count) {
    const int n = *count;
    // every thread of the block reaches the append (block-aggregated atomics)
    __shared__ Append2 s_app;
    const int64_t span = ((int64_t)n + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < span; q += (int64_t)gridDim.x * blockDim.x) {
        Vec3 o{}, d{};
        float te = NAN;
        if (q < n) {
            const int id = queue[q];
            o = load3(ps.o, C, id);
            d = load3(ps.d, C, id);
            te = cube_entry(o, d);
            t0[q] = te;
        }
        const bool enters = q < n && !isnan(te);
        int slot, unused;
        block_append2(query_count, enters, query_count, false, &s_app, slot, unused);
        if (q < n) cmap[q] = enters ? slot : -1;
        if (enters) write_query(rays5, C, slot, o, d, te);
    }
}

// kCount (single-network and mesh scenes): network answers through the compaction map, and
// the bounce's hits counted into hits_out.
template <bool kCount>
__global__ void shade_kernel(ddf_render_params p, int64_t C, int bounce, int backend, const int *__restrict__ queue,
                             int *counts, int *__restrict__ next_queue, PathState ps, const float *__restrict__ t0,
                             const float *__restrict__ logit, const float *__restrict__ dist,
                             const float *__restrict__ grad, const float *__restrict__ tq, const int *__restrict__ triq,
                             const float *__restrict__ tris, int64_t m, int *__restrict__ sq, float *__restrict__ srays,
                             float *__restrict__ st0, float *__restrict__ stmax, float *__restrict__ scontrib,
                             float *__restrict__ depth, float *__restrict__ normal,
                             const unsigned long long *__restrict__ best, const int *__restrict__ cmap,
                             int *__restrict__ hits_out) {
    const int n = counts[2 * bounce];
    const Vec3 light = v3(p.light_pos[0], p.light_pos[1], p.light_pos[2]);
    const int64_t hw = (int64_t)p.width * p.height;
    // every thread of the block reaches the append (block-aggregated atomics)
    __shared__ Append2 s_app;
    __shared__ int s_hits;
    int wave_hits = 0;   // kCount: hits among this wave's paths (wave-uniform)
    const int64_t span = ((int64_t)n + blockDim.x - 1) / blockDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < span; q += (int64_t)gridDim.x * blockDim.x) {
        bool hit = false, shadow = false, alive = false;
        int id = 0;
        Vec3 xs{}, l{}, nd{}, contrib{}, thr{};
        float r = 0.f;
        if (q < n) {
            id = queue[q];
            const Vec3 o = load3(ps.o, C, id), d = load3(ps.d, C, id);
            float t = 0.f;
            Vec3 nrm{};
            if (backend != DDF_BACKEND_MESH) {
                int64_t qs = q;   // where the query's answers are
                if (backend == DDF_BACKEND_NET && kCount) {
                    const int c = cmap[q];   // -1: the ray misses the cube and was not queried
                    if (c >= 0) {
                        t = t0[q] + dist[c];
                        hit = logit[c] > 0.f && t >= 0.f;   // a hit needs a non-negative distance
                    }
                    qs = c >= 0 ? c : 0;
                } else if (backend == DDF_BACKEND_NET) {
                    const float te = t0[q];
                    t = te + dist[q];
                    hit = !isnan(te) && logit[q] > 0.f && t >= 0.f;
                } else {   // MULTI: nearest instance hit, its distance and world-space gradient
                    hit = best[q] != ~0ull;
                    t = dist[q];
                }
                const Vec3 g = load3(grad, C, qs);
                const float gn = sqrtf(dot(g, g)), gd = dot(g, d);
                const float kappa = gd > 0.f ? -1.f : 1.f;   // Eq. 3: n . d < 0
                nrm = gn > 0.f ? (kappa / gn) * g : (-1.0f / sqrtf(dot(d, d))) * d;
            } else {
                const int tri = triq[q];
                hit = tri >= 0;
                t = tq[q];
                if (hit) {
                    const Vec3 a = v3(tris[tri], tris[m + tri], tris[2 * m + tri]);
                    const Vec3 b = v3(tris[3 * m + tri], tris[4 * m + tri], tris[5 * m + tri]);
                    const Vec3 c = v3(tris[6 * m + tri], tris[7 * m + tri], tris[8 * m + tri]);
                    nrm = normalize(cross(b - a, c - a));
                    if (dot(nrm, d) > 0.f) nrm = -1.f * nrm;
                }
            }
            const int pixel = ps.pix[id];
            if (bounce == 0 && ps.smp[id] == 0) {
                if (depth) depth[pixel] = hit ? t : INFINITY;
                if (normal) {
                    normal[pixel] = hit ? nrm.x : 0.f;
                    normal[hw + pixel] = hit ? nrm.y : 0.f;
                    normal[2 * hw + pixel] = hit ? nrm.z : 0.f;
                }
            }
            if (hit) {
                const Vec3 x = o + t * d;
                xs = x + p.eps * nrm;
                const Vec3 lv = light - xs;
                const float r2 = dot(lv, lv);
                r = sqrtf(r2);
                l = (1.0f / r) * lv;
                const float cosl = dot(nrm, l);
                thr = load3(ps.thr, C, id);
                if (cosl > 0.f) {
                    shadow = true;
                    const float k = cosl / (kPi * r2);
                    contrib = v3(thr.x * p.albedo[0] * p.light_intensity[0] * k, thr.y * p.albedo[1] * p.light_intensity[1] * k,
                                 thr.z * p.albedo[2] * p.light_intensity[2] * k);
                }
                if (bounce < p.bounces - 1) {
                    const uint64_t key = path_key(p.seed, (uint64_t)pixel, (uint64_t)ps.smp[id]);
                    const float u1 = uniform01(key, bounce, 2), u2 = uniform01(key, bounce, 3);
                    const float rr = sqrtf(u1), ang = kTwoPi * u2;
                    const float lx = rr * cosf(ang), ly = rr * sinf(ang), lz = sqrtf(fmaxf(0.f, 1.f - u1));
                    // orthonormal basis around the normal (Duff et al. 2017)
                    const float sign = nrm.z >= 0.f ? 1.f : -1.f;
                    const float aa = -1.0f / (sign + nrm.z);
                    const float bb = nrm.x * nrm.y * aa;
                    const Vec3 b1 = v3(1.f + sign * nrm.x * nrm.x * aa, sign * bb, -sign * nrm.x);
                    const Vec3 b2 = v3(bb, sign + nrm.y * nrm.y * aa, -nrm.y);
                    nd = lx * b1 + ly * b2 + lz * nrm;
                    Vec3 tn = v3(thr.x * p.albedo[0], thr.y * p.albedo[1], thr.z * p.albedo[2]);
                    alive = true;
                    if (bounce >= p.rr_start) {
                        const float qs = fminf(0.95f, fmaxf(tn.x, fmaxf(tn.y, tn.z)));
                        if (uniform01(key, bounce, 4) >= qs) alive = false;
                        else tn = (1.0f / qs) * tn;
                    }
                    if (alive) {
                        store3(ps.o, C, id, xs);
                        store3(ps.d, C, id, nd);
                        store3(ps.thr, C, id, tn);
                    }
                }
            }
        }
        if constexpr (kCount) wave_hits += (int)__popcll(__ballot(hit));
        int sslot, nslot;
        block_append2(&counts[2 * bounce + 1], shadow, &counts[2 * (bounce + 1)], alive, &s_app, sslot, nslot);
        if (shadow) {
            sq[sslot] = id;
            stmax[sslot] = r;
            store3(scontrib, C, sslot, contrib);
            if (backend == DDF_BACKEND_NET) {
                const float te = cube_entry(xs, l);
                st0[sslot] = te;
                write_query(srays, C, sslot, xs, l, te);
            } else {   // world-space shadow ray: mesh labeller or per-instance culling
                store3(srays, C, sslot, xs);
                store3(srays + 3 * C, C, sslot, l);
            }
        }
        if (alive) next_queue[nslot] = id;
    }
    if constexpr (kCount) {   // the bounce's hits: one LDS atomic per wave, one global atomic per block
        if (threadIdx.x == 0) s_hits = 0;
        __syncthreads();
        if ((threadIdx.x & 63) == 0 && wave_hits) atomicAdd(&s_hits, wave_hits);
        __syncthreads();
        if (threadIdx.x == 0 && s_hits) atomicAdd(hits_out, s_hits);
    }
}

__global__ void resolve_kernel(int64_t C, int bounce, int backend, const int *__restrict__ counts,
                               const int *__restrict__ sq, const float *__restrict__ st0,
                               const float *__restrict__ stmax, const float *__restrict__ scontrib,
                               const float *__restrict__ slogit, const float *__restrict__ sdist,
                               const float *__restrict__ st, const int *__restrict__ occl, float *__restrict__ L) {
    const int n = counts[2 * bounce + 1];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        bool occluded;
        if (backend == DDF_BACKEND_NET) {
            const float te = st0[q];
            const float t = te + sdist[q];
            occluded = !isnan(te) && slogit[q] > 0.f && t >= 0.f && t < stmax[q];
        } else if (backend == DDF_BACKEND_MULTI) {
            occluded = occl[q] != 0;
        } else {
            occluded = st[q] < stmax[q];
        }
        if (occluded) continue;
        const int id = sq[q];
        L[id] += scontrib[q];
        L[C + id] += scontrib[C + q];
        L[2 * C + id] += scontrib[2 * C + q];
    }
}

__global__ void accumulate_kernel(int64_t hw, int S, int64_t C, const float *__restrict__ L, float *__restrict__ img) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < hw; p += (int64_t)gridDim.x * blockDim.x) {
        float a = 0.f, b = 0.f, c = 0.f;
        for (int s = 0; s < S; ++s) {
            const int64_t id = p * S + s;
            a += L[id];
            b += L[C + id];
            c += L[2 * C + id];
        }
        img[p] += a;
        img[hw + p] += b;
        img[2 * hw + p] += c;
    }
}

__global__ void scale_kernel(float *img, int64_t n, float s) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) img[i] *= s;
}

__global__ void fill_kernel(float *img, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) img[i] = v;
}

// Per bounce: paths entering it (stats[b]) and shadow rays it traced (stats[bounces + b]).
__global__ void stats_kernel(const int *counts, int bounces, uint32_t *stats) {
    const int b = threadIdx.x;
    if (b < bounces) {
        stats[b] += (uint32_t)counts[2 * b];
        stats[bounces + b] += (uint32_t)counts[2 * b + 1];
    }
}

// Single-network and mesh scenes, per bounce: its hits (xstats[b]) and the rays of its
// nearest-hit pass (xstats[bounces + b]: a network scene queries the rays that enter the
// cube, the labeller traces them all).
__global__ void xstats_kernel(const int *counts, const int *xcounts, int bounces, int backend, uint32_t *xstats) {
    const int b = threadIdx.x;
    if (b < bounces) {
        xstats[b] += (uint32_t)xcounts[b];
        xstats[bounces + b] += (uint32_t)(backend == DDF_BACKEND_NET ? xcounts[bounces + b] : counts[2 * b]);
    }
}


// Rays of a queue (main: path ids through `queue`; shadow: rows of `rays6`) against every
// instance's cube.  Pass 0 counts (ray, instance) pairs per instance; pass 1 writes them,
// grouped by instance (and so by network: instances are ordered by network).  Each block
// owns a contiguous range of the queue and aggregates in LDS, so the global counters see
// one atomic per block and instance (per-wave atomics on the same few counters serialised
// in L2).  Both passes run the same grid, so each block covers the same range in both: pass 0
// keeps its per-instance counts, from which pass 1 reserves its slots before its one culling
// sweep that writes.
constexpr int kCullBlock = 256;

template <bool kScatter>
__global__ __launch_bounds__(kCullBlock) void cull_kernel(int64_t C, const int *__restrict__ queue,
                                                          const int *__restrict__ count, const float *__restrict__ po,
                                                          const float *__restrict__ pd,
                                                          const InstDev *__restrict__ inst, int n_inst, MultiCounts mc,
                                                          PairBufs pb, int64_t P) {
    __shared__ InstDev s_inst[kMaxInstances];
    __shared__ int s_cnt[kMaxInstances], s_base[kMaxInstances];
    for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
        s_inst[i] = inst[i];
        s_cnt[i] = 0;
    }
    __syncthreads();
    const int n = *count;
    // contiguous range of this block, a multiple of 64 rays long
    const int64_t per = ((((int64_t)n + gridDim.x - 1) / gridDim.x) + 63) / 64 * 64;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min<int64_t>(lo + per, n);
    const int64_t span = lo < hi ? (hi - lo + 63) / 64 * 64 : 0;   // whole waves: ballots see 64 lanes
    auto sweep = [&](bool write) {
        for (int64_t k = threadIdx.x; k < span; k += blockDim.x) {
            const int64_t q = lo + k;
            const bool live = q < hi;
            Vec3 o{}, d{};
            if (live) {
                const int64_t src = queue ? (int64_t)queue[q] : q;
                o = load3(po, C, src);
                d = load3(pd, C, src);
            }
            for (int i = 0; i < n_inst; ++i) {
                // A ray whose line passes farther than r from T, or that starts outside the
                // sphere heading away from it, cannot enter the cube; every other ray takes
                // the exact test (NaN arguments reject nothing).  The line test's margin grows
                // with |c|^2: the rounding of |c x d|^2 is below 1e-6 |c|^2 |d|^2.
                const InstDev &in = s_inst[i];
                const Vec3 c = v3(in.T[0], in.T[1], in.T[2]) - o;
                const Vec3 x = cross(c, d);
                const float cc = dot(c, c);
                const bool away = dot(x, x) > (in.r2 + 4e-6f * cc) * dot(d, d) || (cc > in.r2 && dot(c, d) < 0.f);
                Vec3 oo{}, dd{};
                float te = NAN;
                if (live && !away) {
                    to_object(in, o, d, oo, dd);
                    te = cube_entry(oo, dd);
                }
                const bool want = !isnan(te);
                if (!write) {
                    const uint64_t mask = __ballot(want);
                    if ((threadIdx.x & 63) == 0 && mask) atomicAdd(&s_cnt[i], (int)__popcll(mask));
                } else {
                    const int slot = append(&s_cnt[i], want);   // LDS counter of this block
                    if (want) {
                        const int64_t p = (int64_t)s_base[i] + slot;
                        pb.q[p] = (int)q;
                        pb.inst[p] = i;
                        pb.t0[p] = te;
                        write_query(pb.rays5, P, p, oo, dd, te);
                    }
                }
            }
        }
    };
    int *const bcount = mc.block_count + (int64_t)blockIdx.x * kMaxInstances;
    if constexpr (!kScatter) {
        sweep(false);
        __syncthreads();
        for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
            bcount[i] = s_cnt[i];
            if (s_cnt[i]) atomicAdd(&mc.inst_count[i], s_cnt[i]);
        }
    } else {
        for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
            const int c = bcount[i];
            s_base[i] = mc.inst_off[i] + (c ? atomicAdd(&mc.inst_cursor[i], c) : 0);
        }
        __syncthreads();
        sweep(true);
    }
}

// Exclusive scan of the per-instance counts; per-network segments; cursor reset; stats.
struct NetMap {
    int user[2 * kMaxNets];   // reordered network index -> caller's index
};

__global__ void pair_scan_kernel(int n_inst, const InstDev *__restrict__ inst, int n_nets, MultiCounts mc,
                                 uint32_t *net_stats, NetMap map) {
    if (threadIdx.x != 0) return;
    int off = 0;
    for (int k = 0; k < n_nets; ++k) {
        mc.seg_offset[k] = off;
        mc.seg_count[k] = 0;
    }
    for (int i = 0; i < n_inst; ++i) {
        mc.inst_off[i] = off;
        mc.inst_cursor[i] = 0;
        mc.seg_count[inst[i].net] += mc.inst_count[i];
        off += mc.inst_count[i];
    }
    for (int k = 0, o = 0; k < n_nets; ++k) {
        mc.seg_offset[k] = o;
        o += mc.seg_count[k];
        if (net_stats) net_stats[map.user[k]] += (uint32_t)mc.seg_count[k];
    }
    *mc.total = off;
}

__global__ void zero_ints_kernel(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void init_best_kernel(const int *__restrict__ count, unsigned long long *best, int *occl) {
    const int n = *count;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        if (best) best[q] = ~0ull;
        if (occl) occl[q] = 0;
    }
}

// Nearest hit over instances: 64-bit key (t bits << 32 | instance) minimised per ray.
__device__ inline unsigned long long hit_key(float t, int inst) {
    return ((unsigned long long)__float_as_uint(t) << 32) | (unsigned)inst;
}

__global__ void merge_kernel(const int *__restrict__ total, PairBufs pb, unsigned long long *best) {
    const int n = *total;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const float t = pb.t0[p] + pb.dist[p];
        if (pb.logit[p] > 0.f && t >= 0.f) atomicMin(&best[pb.q[p]], hit_key(t, pb.inst[p]));
    }
}

// The winning pair of each ray writes its distance and its gradient in world space
// (d dist / d x_world = R d dist / d x_object for x_object = R^T (x_world - T)).
__global__ void select_kernel(int64_t C, const int *__restrict__ total, PairBufs pb, int64_t P,
                              const InstDev *__restrict__ inst, const unsigned long long *__restrict__ best,
                              float *__restrict__ hit_t, float *__restrict__ hit_g) {
    const int n = *total;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const float t = pb.t0[p] + pb.dist[p];
        if (!(pb.logit[p] > 0.f && t >= 0.f)) continue;
        const int q = pb.q[p], i = pb.inst[p];
        if (hit_key(t, i) != best[q]) continue;
        const InstDev &in = inst[i];
        const Vec3 g = load3(pb.grad, P, p);
        hit_t[q] = t;
        store3(hit_g, C, q, v3(in.R[0] * g.x + in.R[1] * g.y + in.R[2] * g.z, in.R[3] * g.x + in.R[4] * g.y + in.R[5] * g.z,
                              in.R[6] * g.x + in.R[7] * g.y + in.R[8] * g.z));
    }
}

__global__ void occlude_kernel(const int *__restrict__ total, PairBufs pb, const float *__restrict__ stmax, int *occl) {
    const int n = *total;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const float t = pb.t0[p] + pb.dist[p];
        const int q = pb.q[p];
        if (pb.logit[p] > 0.f && t >= 0.f && t < stmax[q]) occl[q] = 1;
    }
}

int chunk_spp(const ddf_render_params &p, int n_inst) {
    if (p.spp_chunk > 0) return std::min(p.spp_chunk, p.spp);
    const int64_t hw = (int64_t)p.width * p.height;
    const int64_t budget = n_inst > 0 ? ((int64_t)1 << 26) / n_inst : ((int64_t)1 << 24);   // paths (pairs) per chunk
    return (int)std::max<int64_t>(1, std::min<int64_t>(p.spp, budget / hw));
}

int scene_instances(const ddf_scene *scene) { return scene && scene->backend == DDF_BACKEND_MULTI ? scene->n_instances : 0; }

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

ddf_status check_net_for_render(const ddf_net *net, const char *who) {
    DDF_REQUIRE(net && net->packed, DDF_ERR_INVALID_ARG, "%s: NULL network", who);
    DDF_REQUIRE(net->precision == DDF_PREC_FP32 || net->precision == DDF_PREC_BF16, DDF_ERR_UNSUPPORTED,
                "%s: the network backends need float32 or bfloat16 networks (normals)", who);
    DDF_REQUIRE((net->width == 128 || net->width == 256) && net->depth >= 1 && net->depth <= 8, DDF_ERR_UNSUPPORTED,
                "%s: unsupported network shape", who);
    return DDF_OK;
}

ddf_status check_scene(const ddf_scene *scene) {
    DDF_REQUIRE(scene, DDF_ERR_INVALID_ARG, "ddf_render: NULL scene");
    if (scene->backend == DDF_BACKEND_MESH) {
        DDF_REQUIRE(scene->m >= 0 && (scene->m == 0 || scene->tris), DDF_ERR_INVALID_ARG, "ddf_render: bad mesh");
        return DDF_OK;
    }
    if (scene->backend == DDF_BACKEND_NET) return check_net_for_render(scene->net, "ddf_render");
    DDF_REQUIRE(scene->backend == DDF_BACKEND_MULTI, DDF_ERR_INVALID_ARG, "ddf_render: unknown backend %d", scene->backend);
    DDF_REQUIRE(scene->n_nets >= 1 && scene->nets && scene->n_instances >= 1 && scene->instances &&
                    scene->n_instances <= kMaxInstances,
                DDF_ERR_INVALID_ARG, "ddf_render: a multi-object scene needs 1..%d instances and networks", kMaxInstances);
    int per_width[2] = {0, 0};
    for (int k = 0; k < scene->n_nets; ++k) {
        if (ddf_status st = check_net_for_render(&scene->nets[k], "ddf_render (multi)")) return st;
        DDF_REQUIRE(scene->nets[k].precision == scene->nets[0].precision, DDF_ERR_UNSUPPORTED,
                    "ddf_render: all networks of a scene need the same precision");
        ++per_width[scene->nets[k].width == 128 ? 0 : 1];
    }
    DDF_REQUIRE(per_width[0] <= kMaxNets && per_width[1] <= kMaxNets, DDF_ERR_UNSUPPORTED,
                "ddf_render: at most %d networks of each width", kMaxNets);
    for (int i = 0; i < scene->n_instances; ++i)
        DDF_REQUIRE(scene->instances[i].net >= 0 && scene->instances[i].net < scene->n_nets, DDF_ERR_INVALID_ARG,
                    "ddf_render: instance %d names network %d", i, scene->instances[i].net);
    return DDF_OK;
}

// Networks ordered by width (128 first), instances ordered by network: every width group and
// every network's (ray, instance) pairs are then contiguous.
struct MultiPlan {
    int n_nets = 0, n_inst = 0;
    int order[2 * kMaxNets];          // reordered index -> caller's network index
    int group_first[2] = {0, 0}, group_size[2] = {0, 0}, group_width[2] = {128, 256};
    std::vector<InstDev> inst;
};

MultiPlan make_plan(const ddf_scene *scene) {
    MultiPlan mp;
    mp.n_nets = scene->n_nets;
    mp.n_inst = scene->n_instances;
    int pos[2 * kMaxNets];
    int k2 = 0;
    for (int g = 0; g < 2; ++g) {
        mp.group_first[g] = k2;
        for (int k = 0; k < scene->n_nets; ++k)
            if (scene->nets[k].width == mp.group_width[g]) {
                pos[k] = k2;
                mp.order[k2++] = k;
            }
        mp.group_size[g] = k2 - mp.group_first[g];
    }
    std::vector<int> idx(scene->n_instances);
    for (int i = 0; i < scene->n_instances; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return pos[scene->instances[a].net] < pos[scene->instances[b].net]; });
    for (int i : idx) {
        InstDev d{};
        for (int j = 0; j < 9; ++j) d.R[j] = scene->instances[i].R[j];
        for (int j = 0; j < 3; ++j) d.T[j] = scene->instances[i].T[j];
        d.net = pos[scene->instances[i].net];
        // a rotation (R R^T = I) moves the cube [-1, 1]^3 within sqrt(3) of T; the radius is
        // widened by half a percent to cover rounding, and any other R culls exactly only
        double err = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double e = a == b ? -1.0 : 0.0;
                for (int k = 0; k < 3; ++k) e += (double)d.R[3 * a + k] * d.R[3 * b + k];
                err = std::max(err, std::fabs(e));
            }
        d.r2 = err <= 1e-4 ? 3.0f * 1.01f : INFINITY;
        mp.inst.push_back(d);
    }
    return mp;
}

// Nearest hit (main) or occlusion (shadow) of a queue of world rays against every instance.
ddf_status multi_query(const ddf_scene *scene, const MultiPlan &mp, RenderWs &w, int64_t C, const int *queue,
                       const int *count, const float *po, const float *pd, bool shadow, uint32_t *net_stats,
                       const float *stmax, hipStream_t s) {
    const unsigned gC = grid_for(C), gP = grid_for(w.P);
    NetMap map{};
    for (int k = 0; k < mp.n_nets; ++k) map.user[k] = mp.order[k];
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(kMaxInstances), 0, s, w.mc.inst_count, kMaxInstances);
    // a few thousand rays per block (a tuning knob): one global atomic per block and instance
    const int64_t rpb = tuning(DDF_TUNE_CULL_RAYS_PER_BLOCK);
    const unsigned gCull = (unsigned)std::max<int64_t>(1, std::min<int64_t>((C + rpb - 1) / rpb, kMaxCullBlocks));
    hipLaunchKernelGGL(cull_kernel<false>, dim3(gCull), dim3(kCullBlock), 0, s, C, queue, count, po, pd, w.inst, mp.n_inst, w.mc, w.pb, w.P);
    hipLaunchKernelGGL(pair_scan_kernel, dim3(1), dim3(64), 0, s, mp.n_inst, w.inst, mp.n_nets, w.mc, net_stats, map);
    hipLaunchKernelGGL(cull_kernel<true>, dim3(gCull), dim3(kCullBlock), 0, s, C, queue, count, po, pd, w.inst, mp.n_inst, w.mc, w.pb, w.P);
    if (ddf_status st = launch_status("ddf_render_wavefront (instance culling)")) return st;
    for (int g = 0; g < 2; ++g) {
        if (mp.group_size[g] == 0) continue;
        GradArgs a{};
        a.rays = w.pb.rays5;
        a.n = w.P;
        a.g_dist_in = w.pb.ones;
        a.logit_out = w.pb.logit;
        a.dist_out = w.pb.dist;
        a.g_rays = shadow ? nullptr : w.pb.grad;
        a.forward_only = shadow;
        a.grad_hits_only = true;   // normals are read for hits only
        a.n_nets = mp.group_size[g];
        a.depth = 1;
        for (int j = 0; j < mp.group_size[g]; ++j) {
            const ddf_net &net = scene->nets[mp.order[mp.group_first[g] + j]];
            a.blobs[j] = (const uint8_t *)net.packed;
            a.depths[j] = net.depth;
            a.depth = std::max(a.depth, net.depth);
        }
        a.blob = a.blobs[0];
        a.seg_offset = w.mc.seg_offset + mp.group_first[g];
        a.seg_count = w.mc.seg_count + mp.group_first[g];
        if (ddf_status st = grad_dispatch_multi(mp.group_width[g], scene->nets[0].precision, a, s)) return st;
    }
    if (!shadow) {
        hipLaunchKernelGGL(init_best_kernel, dim3(gC), dim3(256), 0, s, count, w.best, (int *)nullptr);
        hipLaunchKernelGGL(merge_kernel, dim3(gP), dim3(256), 0, s, w.mc.total, w.pb, w.best);
        hipLaunchKernelGGL(select_kernel, dim3(gP), dim3(256), 0, s, C, w.mc.total, w.pb, w.P, w.inst, w.best, w.hit_t,
                           w.hit_g);
    } else {
        hipLaunchKernelGGL(init_best_kernel, dim3(gC), dim3(256), 0, s, count, (unsigned long long *)nullptr, w.occl);
        hipLaunchKernelGGL(occlude_kernel, dim3(gP), dim3(256), 0, s, w.mc.total, w.pb, stmax, w.occl);
    }
    return launch_status("ddf_render_wavefront (multi-object query)");
}

}  // namespace
}  // namespace ddf

using namespace ddf;

extern "C" ddf_status ddf_render_workspace_size(const ddf_scene *scene, const ddf_render_params *p, size_t *bytes) {
    DDF_REQUIRE(p && bytes, DDF_ERR_INVALID_ARG, "ddf_render_workspace_size: NULL argument");
    DDF_REQUIRE(p->width > 0 && p->height > 0 && p->spp > 0 && p->bounces > 0 && p->bounces <= 64, DDF_ERR_INVALID_ARG,
                "ddf_render_workspace_size: bad image size, spp or bounces");
    const int n_inst = scene_instances(scene);
    DDF_REQUIRE(n_inst <= kMaxInstances, DDF_ERR_UNSUPPORTED, "ddf_render_workspace_size: too many instances");
    const int64_t C = (int64_t)p->width * p->height * chunk_spp(*p, n_inst);
    DDF_REQUIRE(C * std::max(1, n_inst) < ((int64_t)1 << 31), DDF_ERR_UNSUPPORTED,
                "ddf_render_workspace_size: sample chunk too large");
    *bytes = render_ws(C, p->bounces, n_inst, nullptr).bytes;
    return DDF_OK;
}

extern "C" ddf_status ddf_render_wavefront(const ddf_scene *scene, const ddf_render_params *p, float *radiance,
                                           float *depth, float *normal, uint32_t *stats, void *ws, size_t ws_bytes,
                                           ddf_stream stream) {
    DDF_REQUIRE(scene && p && radiance, DDF_ERR_INVALID_ARG, "ddf_render_wavefront: NULL argument");
    size_t need = 0;
    if (ddf_status st = ddf_render_workspace_size(scene, p, &need)) return st;
    DDF_REQUIRE(ws && ws_bytes >= need, DDF_ERR_WORKSPACE, "ddf_render_wavefront: workspace of %zu bytes needed", need);
    if (ddf_status st = check_scene(scene)) return st;
    DDF_REQUIRE(p->rr_start >= 0 && p->eps >= 0.f && p->vfov_deg > 0.f && p->vfov_deg < 180.f, DDF_ERR_INVALID_ARG,
                "ddf_render_wavefront: bad rr_start, eps or field of view");
    hipStream_t s = as_stream(stream);
    const int n_inst = scene_instances(scene);
    const bool multi = n_inst > 0;
    const int S = chunk_spp(*p, n_inst);
    const int64_t hw = (int64_t)p->width * p->height;
    const int64_t C = hw * S;
    RenderWs w = render_ws(C, p->bounces, n_inst, ws);
    const Cam cam = make_cam(*p);
    const int ncounts = 2 * p->bounces + 4;
    MultiPlan mp;
    if (multi) {
        mp = make_plan(scene);
        for (int first = 0; first < n_inst; first += kInstChunk) {
            InstChunk c{};
            const int cnt = std::min(kInstChunk, n_inst - first);
            for (int j = 0; j < cnt; ++j) c.v[j] = mp.inst[first + j];
            hipLaunchKernelGGL(inst_table_kernel, dim3(1), dim3(kInstChunk), 0, s, c, first, cnt, w.inst);
        }
        hipLaunchKernelGGL(fill_kernel, dim3(grid_for(w.P)), dim3(256), 0, s, w.pb.ones, w.P, 1.0f);
    }
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(3 * hw)), dim3(256), 0, s, radiance, 3 * hw, 0.f);
    const int64_t nstats = (int64_t)p->bounces * (multi ? 2 + scene->n_nets : 4);
    if (stats) hipLaunchKernelGGL(fill_kernel, dim3(grid_for(nstats)), dim3(256), 0, s, (float *)stats, nstats, 0.f);
    for (int base = 0; base < p->spp; base += S) {
        const int Sc = std::min(S, p->spp - base);
        const int64_t Cc = hw * Sc;
        hipLaunchKernelGGL(raygen_kernel, dim3(grid_for(Cc)), dim3(256), 0, s, *p, cam, Cc, base, Sc, w.ps, w.qa,
                           w.counts, ncounts, w.ones, depth, normal);
        if (!multi) hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(128), 0, s, w.xcounts, 2 * p->bounces);
        // path-state arrays use the chunk's own stride Cc (== C except in a short last chunk)
        PathState ps = w.ps;
        int *q = w.qa, *qn = w.qb;
        for (int b = 0; b < p->bounces; ++b) {
            const int *cnt = w.counts + 2 * b;
            const float *qdist = w.dist, *qgrad = w.grad;
            if (scene->backend == DDF_BACKEND_NET) {
                int *qcnt = w.xcounts + p->bounces + b;   // this bounce's queries
                hipLaunchKernelGGL(prep_kernel, dim3(grid_for(Cc)), dim3(256), 0, s, Cc, q, cnt, ps, w.rays5, w.t0,
                                   w.cmap, qcnt);
                GradArgs a{};
                a.blob = (const uint8_t *)scene->net->packed;
                a.depth = scene->net->depth;
                a.rays = w.rays5;
                a.n = Cc;
                a.count_dev = qcnt;
                a.g_dist_in = w.ones;
                a.logit_out = w.logit;
                a.dist_out = w.dist;
                a.g_rays = w.grad;
                a.grad_hits_only = true;   // normals are read for hits only
                if (ddf_status st = grad_dispatch(scene->net, a, false, s)) return st;
            } else if (multi) {
                if (ddf_status st = multi_query(scene, mp, w, Cc, q, cnt, ps.o, ps.d, false,
                                                stats ? stats + 2 * p->bounces + (int64_t)b * scene->n_nets : nullptr,
                                                nullptr, s))
                    return st;
                qdist = w.hit_t;
                qgrad = w.hit_g;
            } else {
                if (ddf_status st = label_queue(ps.o, ps.d, Cc, q, cnt, scene->tris, scene->m, 0.f, INFINITY, w.tq, w.triq, s))
                    return st;
            }
            if (multi)
                hipLaunchKernelGGL(shade_kernel<false>, dim3(grid_for(Cc)), dim3(256), 0, s, *p, Cc, b, scene->backend, q,
                                   w.counts, qn, ps, w.t0, w.logit, qdist, qgrad, w.tq, w.triq, scene->tris, scene->m, w.sq,
                                   w.srays, w.st0, w.stmax, w.scontrib, depth, normal, (const unsigned long long *)w.best,
                                   (const int *)nullptr, (int *)nullptr);
            else
                hipLaunchKernelGGL(shade_kernel<true>, dim3(grid_for(Cc)), dim3(256), 0, s, *p, Cc, b, scene->backend, q,
                                   w.counts, qn, ps, w.t0, w.logit, qdist, qgrad, w.tq, w.triq, scene->tris, scene->m, w.sq,
                                   w.srays, w.st0, w.stmax, w.scontrib, depth, normal, (const unsigned long long *)w.best,
                                   (const int *)w.cmap, w.xcounts + b);
            if (ddf_status st = launch_status("ddf_render_wavefront (shade)")) return st;
            const int *scnt = w.counts + 2 * b + 1;
            if (scene->backend == DDF_BACKEND_NET) {
                if (ddf_status st = forward_dispatch(scene->net, w.srays, Cc, scnt, w.slogit, w.sdist, nullptr, s)) return st;
            } else if (multi) {
                if (ddf_status st = multi_query(scene, mp, w, Cc, nullptr, scnt, w.srays, w.srays + 3 * Cc, true, nullptr,
                                                w.stmax, s))
                    return st;
            } else {
                if (ddf_status st = label_queue(w.srays, w.srays + 3 * Cc, Cc, nullptr, scnt, scene->tris, scene->m, 0.f,
                                                INFINITY, w.st, w.stri, s))
                    return st;
            }
            hipLaunchKernelGGL(resolve_kernel, dim3(grid_for(Cc)), dim3(256), 0, s, Cc, b, scene->backend, w.counts, w.sq,
                               w.st0, w.stmax, w.scontrib, w.slogit, w.sdist, w.st, (const int *)w.occl, ps.L);
            std::swap(q, qn);
        }
        hipLaunchKernelGGL(accumulate_kernel, dim3(grid_for(hw)), dim3(256), 0, s, hw, Sc, Cc, ps.L, radiance);
        if (stats) hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(64), 0, s, w.counts, p->bounces, stats);
        if (stats && !multi)
            hipLaunchKernelGGL(xstats_kernel, dim3(1), dim3(64), 0, s, w.counts, w.xcounts, p->bounces, scene->backend,
                               stats + 2 * p->bounces);
        if (ddf_status st = launch_status("ddf_render_wavefront")) return st;
    }
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(3 * hw)), dim3(256), 0, s, radiance, 3 * hw, 1.0f / (float)p->spp);
    return launch_status("ddf_render_wavefront");
}
