"""Path-tracer oracle (Fig. 1): camera rays, nearest hit, shading normal, next-event
estimation towards a point light, cosine-weighted Lambertian scattering and
Russian roulette, with either the triangle mesh or the network as the scene.

Test infrastructure only (see the package docstring).

The paper describes the renderer only as a path tracer whose nearest-triangle
search is replaced by the distance field, with normals from the field's
gradient (Sec. I, Sec. IV, Fig. 1).  The readings used here:

* pinhole camera; pixel centre at 1 sample per pixel, otherwise a jitter from
  random dimensions 0 and 1;
* network queries start at the entry point of the domain cube [-1,1]^3 when
  the ray origin lies outside it; hit distance = entry offset + predicted
  distance; hit <=> logit > 0 and that distance >= 0;
* normal: mesh face normal, or Eq. 3 applied to d(dist)/d(origin); flipped so
  that n . d < 0;
* next-event estimation: a shadow ray from x + eps n to the light; visible
  when nothing is hit before the light; contribution
  throughput * (albedo / pi) * I * max(0, n . l) / r^2;
* scattering: Malley's method (r = sqrt(u1), angle 2 pi u2) in the
  orthonormal basis of Duff et al. (2017); throughput *= albedo; the scatter
  is skipped after the last bounce;
* Russian roulette after the scatter of bounce b >= rr_start with survival
  probability q = min(0.95, max channel of throughput), throughput /= q.

Random numbers are counter based: u = (h >> 40) * 2^-24 with
h = H(H(H(H(H(seed) ^ pixel) ^ sample) ^ bounce) ^ dim), where H(x) is the
first output of a SplitMix64 generator (Steele, Lea and Flood, 2014) whose
state is x.  Dimensions: 0, 1 pixel jitter; 2, 3 scatter; 4 roulette.
"""
import numpy as np

from . import geometry, mlp

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64_mix(z):
    """SplitMix64 output function applied to a state (Python ints)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64_stream(seed, n):
    """The first ``n`` outputs of SplitMix64 seeded with ``seed`` (pinned by published values)."""
    out, s = [], seed & M64
    for _ in range(n):
        s = (s + GOLDEN) & M64
        out.append(splitmix64_mix(s))
    return out


def _h(x):
    return splitmix64_mix((x + GOLDEN) & M64)


def _h_np(x):
    """Vectorised H over uint64 arrays (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def path_keys(seed, pixel, sample):
    """Per-path key H(H(H(seed) ^ pixel) ^ sample) for uint64 arrays of pixel and sample."""
    k = _h_np(np.uint64(_h(seed)) ^ pixel.astype(np.uint64))
    return _h_np(k ^ sample.astype(np.uint64))


def uniform(path_key, bounce, dim):
    """Counter-based uniform in [0, 1) (exact float32 value, returned as float64)."""
    k = _h_np(path_key ^ np.uint64(bounce))
    k = _h_np(k ^ np.uint64(dim))
    return (k >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def uniform_scalar(seed, pixel, sample, bounce, dim):
    k = _h(_h(_h(_h(_h(seed) ^ pixel) ^ sample) ^ bounce) ^ dim)
    return (k >> 40) * 2.0 ** -24


def camera_rays(cfg, pixel, sample, keys):
    """Pinhole camera rays for the given pixel indices (row 0 at the top)."""
    cam = cfg.camera
    W, H = cfg.width, cfg.height
    eye = np.asarray(cam.eye, dtype=np.float64)
    f = np.asarray(cam.target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(cam.up, dtype=np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = np.tan(np.radians(cam.vfov_deg) * 0.5)
    px = (pixel % W).astype(np.float64)
    py = (pixel // W).astype(np.float64)
    if cfg.spp == 1:
        jx = np.full(px.shape, 0.5)
        jy = np.full(px.shape, 0.5)
    else:
        jx = uniform(keys, 0, 0)
        jy = uniform(keys, 0, 1)
    sx = (2.0 * (px + jx) / W - 1.0) * th * (W / H)
    sy = (1.0 - 2.0 * (py + jy) / H) * th
    d = f[:, None] + sx[None] * r[:, None] + sy[None] * u[:, None]
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    o = np.repeat(eye[:, None], px.size, axis=1)
    return o, d


def onb_duff(n):
    """Orthonormal basis (b1, b2) around unit normals ``n`` [3, N] (Duff et al. 2017)."""
    sign = np.where(n[2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[2])
    b = n[0] * n[1] * a
    b1 = np.stack([1.0 + sign * n[0] * n[0] * a, sign * b, -sign * n[0]])
    b2 = np.stack([b, sign + n[1] * n[1] * a, -n[1]])
    return b1, b2


class MeshScene:
    """Scene backend: nearest hit by brute force over a triangle soup (oracle geometry)."""

    def __init__(self, tris, amb_tol=1e-6):
        self.tris = np.asarray(tris)
        self.fn = geometry.face_normals(self.tris)
        self.amb_tol = amb_tol

    def intersect(self, o, d, t_max):
        r = geometry.nearest_hit(o, d, self.tris, 0.0, t_max, amb_tol=self.amb_tol)
        hit = r["tri"] >= 0
        n = self.fn[:, np.maximum(r["tri"], 0)]
        margin_ok = ~r["ambiguous"]
        return hit, r["t"], n, margin_ok

    def occluded(self, o, d, t_max):
        r = geometry.nearest_hit(o, d, self.tris, 0.0, t_max, amb_tol=self.amb_tol)
        return r["tri"] >= 0, ~r["ambiguous"]


class NetworkScene:
    """Scene backend: the network, queried from the domain-cube entry point."""

    def __init__(self, params, width, depth, logit_margin=1e-4, precision="fp64"):
        """precision "bf16": the network is evaluated as ``mlp.forward_bf16`` and its input
        gradient as ``mlp.backward_input_bf16`` (bfloat16 operands, float64 sums)."""
        self.params = params
        self.width = width
        self.depth = depth
        self.margin = logit_margin
        self.bf16 = precision == "bf16"

    def _query(self, o, d):
        t_in, t_out, inbox = geometry.cube_entry(o, d)
        t0 = np.maximum(t_in, 0.0)
        q = o + t0[None] * d
        theta, phi = geometry.angles_from_dirs(d)
        rays = np.concatenate([q, theta[None], phi[None]])
        fwd = mlp.forward_bf16 if self.bf16 else mlp.forward
        logit, dist = fwd(self.params, self.width, self.depth, rays)
        t = t0 + dist
        hit = inbox & (logit > 0.0) & (t >= 0.0)   # a hit needs a non-negative distance
        robust = ~inbox | ((np.abs(logit) > self.margin) & (np.abs(t) > self.margin))
        return hit, t, rays, robust

    def intersect(self, o, d, t_max):
        hit, t, rays, robust = self._query(o, d)
        n = rays.shape[1]
        if self.bf16:
            g = mlp.backward_input_bf16(self.params, self.width, self.depth, rays, np.zeros(n), np.ones(n))
        else:
            g, _ = mlp.backward(self.params, self.width, self.depth, rays, np.zeros(n), np.ones(n))
        # a nearly vanishing gradient leaves the normal (and every later bounce) undecided
        gn = np.linalg.norm(g[0:3], axis=0)
        robust = robust & ~(hit & (gn < self.margin * 10.0))
        return hit, t, g[0:3], robust

    def occluded(self, o, d, t_max):
        hit, t, _, robust = self._query(o, d)
        # also undecided when the predicted hit lies at the light within the margin
        robust = robust & ~(hit & (np.abs(t - t_max) <= self.margin * (1.0 + np.abs(t_max))))
        return hit & (t < t_max), robust


def render(scene, cfg, pixels=None):
    """Render ``cfg`` (a ``synthetic.RenderConfig``) with a scene backend.

    Returns a dict: ``radiance`` [3, H, W] (mean over samples), ``depth`` [H, W]
    and ``normal`` [3, H, W] of sample 0's primary hit (depth +inf and normal 0
    on a miss), ``robust`` [H, W] (every query of every sample of the pixel was
    decided away from its threshold), ``active`` per bounce (number of
    paths that entered the bounce), ``queried`` per bounce (rays of the nearest-hit pass: a
    network scene queries only the rays that enter the domain cube, any other scene traces
    them all), ``hits`` per bounce (paths whose query hit) and ``shadow`` per bounce (number
    of shadow rays traced: hits whose normal faces the light).

    ``pixels``: optional flat pixel indices (row * W + column).  Only those pixels
    are traced (every path is independent, so each one is traced exactly as in the
    whole frame) and the per-pixel arrays come back as [3, len] / [len] in that
    order; the per-bounce counts then count the paths of those pixels only.
    """
    W, H, S = cfg.width, cfg.height, cfg.spp
    pix = np.arange(W * H, dtype=np.int64) if pixels is None else np.asarray(pixels, dtype=np.int64)
    npx = pix.size
    P = npx * S
    pid = np.arange(P, dtype=np.int64)
    pixel = pix[pid // S]
    sample = pid % S
    keys = path_keys(cfg.seed, pixel, sample)
    o, d = camera_rays(cfg, pixel, sample, keys)
    albedo = np.asarray(cfg.albedo, dtype=np.float64)[:, None]
    light = np.asarray(cfg.light.position, dtype=np.float64)[:, None]
    inten = np.asarray(cfg.light.intensity, dtype=np.float64)[:, None]
    thr = np.ones((3, P))
    L = np.zeros((3, P))
    alive = np.ones(P, dtype=bool)
    robust = np.ones(P, dtype=bool)
    depth0 = np.full(P, np.inf)
    normal0 = np.zeros((3, P))
    active, queried, hits, shadow = [], [], [], []
    for b in range(cfg.bounces):
        idx = np.nonzero(alive)[0]
        active.append(int(idx.size))
        if idx.size == 0:
            break
        if isinstance(scene, NetworkScene):   # a ray that misses the cube misses the object
            queried.append(int(geometry.cube_entry(o[:, idx], d[:, idx])[2].sum()))
        else:
            queried.append(int(idx.size))
        hit, t, n, ok = scene.intersect(o[:, idx], d[:, idx], np.inf)
        robust[idx] &= ok
        hits.append(int(hit.sum()))
        if b == 0:
            depth0[idx] = np.where(hit, t, np.inf)
        alive[idx[~hit]] = False
        idx, t, n = idx[hit], t[hit], n[:, hit]
        if idx.size == 0:
            break
        dd = d[:, idx]
        if not isinstance(scene, MeshScene):   # network scenes return the distance gradient
            n = mlp.normals(n, dd)
        else:
            n = np.where(np.sum(n * dd, axis=0) > 0.0, -n, n)
        if b == 0:
            normal0[:, idx] = n
        x = o[:, idx] + t[None] * dd
        xs = x + cfg.eps * n
        lv = light - xs
        r2 = np.sum(lv * lv, axis=0)
        r = np.sqrt(r2)
        l = lv / r[None]
        cosl = np.sum(n * l, axis=0)
        lit = cosl > 0.0
        shadow.append(int(lit.sum()))
        vis = np.zeros(idx.size, dtype=bool)
        if lit.any():
            occ, ok = scene.occluded(xs[:, lit], l[:, lit], r[lit])
            vis[lit] = ~occ
            rb = robust[idx]
            rb[lit] &= ok
            robust[idx] = rb
        contrib = thr[:, idx] * (albedo / np.pi) * inten * np.where(vis, cosl, 0.0)[None] / r2[None]
        L[:, idx] += contrib
        if b == cfg.bounces - 1:
            break
        u1 = uniform(keys[idx], b, 2)
        u2 = uniform(keys[idx], b, 3)
        rr = np.sqrt(u1)
        ang = 2.0 * np.pi * u2
        lx, ly, lz = rr * np.cos(ang), rr * np.sin(ang), np.sqrt(np.maximum(0.0, 1.0 - u1))
        b1, b2 = onb_duff(n)
        nd = b1 * lx[None] + b2 * ly[None] + n * lz[None]
        o[:, idx] = xs
        d[:, idx] = nd
        thr[:, idx] *= albedo
        if b >= cfg.rr_start:
            q = np.minimum(0.95, thr[:, idx].max(axis=0))
            die = uniform(keys[idx], b, 4) >= q
            alive[idx[die]] = False
            keep = idx[~die]
            thr[:, keep] /= q[~die][None]
    shape = (H, W) if pixels is None else (npx,)
    rad = L.reshape(3, npx, S).mean(axis=2).reshape((3,) + shape)
    first = pid % S == 0
    return {
        "radiance": rad,
        "depth": depth0[first].reshape(shape),
        "normal": normal0[:, first].reshape((3,) + shape),
        "robust": robust.reshape(npx, S).all(axis=1).reshape(shape),
        "active": active,
        "queried": queried,
        "hits": hits,
        "shadow": shadow,
    }
