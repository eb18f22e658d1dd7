"""Procedural triangle meshes (the stand-ins for the paper's evaluation meshes).

The paper trains on ShapeNet objects, the Stanford bunny and Suzanne (Sec. VI-B);
none of those assets are used here.  Instead the workloads use:

* an icosphere (icosahedron, 1->4 midpoint subdivision, vertices pushed to a
  sphere): subdivision 2 has 162 vertices and 320 triangles;
* a disjoint union of three tori (64 x 40 segments, 5,120 triangles each) and one
  subdivision-4 icosphere (5,120 triangles): 20,480 triangles, unique vertices
  jittered by N(0, 0.005);
* for the multi-object scenes, further unions of tori and spheres whose
  tessellation is chosen to reach a drawn triangle count.

Meshes are returned as ``(vertices float64 [V,3], faces int64 [F,3])`` with
counter-clockwise (outward) winding.  ``tri_soup`` turns a mesh into the
structure-of-arrays float32 buffer the labeller consumes: nine rows
``v0x v0y v0z v1x v1y v1z v2x v2y v2z``, one column per triangle.
"""
import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _icosahedron():
    v = np.array([
        [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
        [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
        [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v / np.linalg.norm(v, axis=1, keepdims=True), f


def icosphere(subdiv=2, radius=0.8, center=(0.0, 0.0, 0.0)):
    """Icosahedron refined ``subdiv`` times by 1->4 midpoint splits, projected to ``radius``."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                p = (np.asarray(verts[a]) + np.asarray(verts[b])) * 0.5
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
    v = np.asarray(verts, dtype=np.float64) * radius + np.asarray(center, dtype=np.float64)
    return v, f


def torus(major, minor, n_major=64, n_minor=40, rotation=None, center=(0.0, 0.0, 0.0)):
    """Torus around the local z axis with ``n_major * n_minor * 2`` triangles."""
    i = np.arange(n_major)
    j = np.arange(n_minor)
    u = 2.0 * np.pi * i / n_major
    w = 2.0 * np.pi * j / n_minor
    uu, ww = np.meshgrid(u, w, indexing="ij")
    ring = major + minor * np.cos(ww)
    v = np.stack([ring * np.cos(uu), ring * np.sin(uu), minor * np.sin(ww)], axis=-1).reshape(-1, 3)
    ii, jj = np.meshgrid(i, j, indexing="ij")
    a = ii * n_minor + jj
    b = ((ii + 1) % n_major) * n_minor + jj
    c = ((ii + 1) % n_major) * n_minor + (jj + 1) % n_minor
    d = ii * n_minor + (jj + 1) % n_minor
    f = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3), np.stack([a, c, d], -1).reshape(-1, 3)])
    if rotation is not None:
        v = v @ np.asarray(rotation, dtype=np.float64).T
    return v + np.asarray(center, dtype=np.float64), f.astype(np.int64)


def union(*meshes):
    """Concatenate meshes (no boolean operation: the parts must not overlap)."""
    vs, fs, off = [], [], 0
    for v, f in meshes:
        vs.append(v)
        fs.append(f + off)
        off += len(v)
    return np.concatenate(vs), np.concatenate(fs)


def jitter_vertices(v, sigma, rng):
    return v + rng.normal(0.0, sigma, size=v.shape)


def _random_rotation(rng):
    """Uniform rotation from a uniform unit quaternion (Shoemake's method)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([
        np.sqrt(1 - u1) * np.sin(2 * np.pi * u2), np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
        np.sqrt(u1) * np.sin(2 * np.pi * u3), np.sqrt(u1) * np.cos(2 * np.pi * u3)])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def _place_disjoint(rng, radii, half=0.97, max_tries=20000):
    """Rejection-sample centres so spheres of ``radii`` are pairwise disjoint and inside the cube
    ``[-half, half]^3``; parts are placed largest first, and the whole placement restarts
    (continuing the same random stream) when a part finds no room."""
    order = np.argsort(-np.asarray(radii), kind="stable")
    for _ in range(50):
        centres = {}
        for k in order:
            r = radii[k]
            if r >= half:
                raise RuntimeError("part larger than the domain")
            for _ in range(max_tries):
                c = rng.uniform(-(half - r), half - r, size=3)
                if all(np.linalg.norm(c - c2) > r + radii[k2] for k2, c2 in centres.items()):
                    centres[k] = c
                    break
            else:
                break
        if len(centres) == len(radii):
            return [centres[k] for k in range(len(radii))]
    return None


def _primitive_union(rng, n_tori, tri_budget_per_part, sphere_subdiv, jitter):
    """Tori with radii U(0.2,0.5)/U(0.05,0.15) plus one sphere U(0.15,0.3), disjoint in the unit ball.

    Draw order: (major, minor) per torus, the sphere radius, placement centres
    (rejection sampling; radii are redrawn when no placement is found), one
    rotation per torus, then the vertex jitter.
    """
    while True:
        majors = rng.uniform(0.2, 0.5, size=n_tori)
        minors = rng.uniform(0.05, 0.15, size=n_tori)
        sphere_r = rng.uniform(0.15, 0.3)
        radii = list(majors + minors) + [sphere_r]
        centres = _place_disjoint(rng, radii)
        if centres is not None:
            break
    parts = []
    for k in range(n_tori):
        nm, nn = tri_budget_per_part
        parts.append(torus(majors[k], minors[k], nm, nn, rotation=_random_rotation(rng), center=centres[k]))
    parts.append(icosphere(sphere_subdiv, sphere_r, centres[-1]))
    v, f = union(*parts)
    return jitter_vertices(v, jitter, rng), f


def training_mesh(seed=1):
    """20,480-triangle mesh: 3 tori (64 x 40 segments) + an icosphere (subdivision 4), jitter N(0, 0.005)."""
    rng = np.random.default_rng(seed)
    return _primitive_union(rng, 3, (64, 40), 4, 0.005)


def multi_object_mesh(seed, tri_lo=2000, tri_hi=50000):
    """One object of the multi-object scene: 1-3 tori + a sphere, about a log-uniform triangle count.

    Draw order: triangle target (log-uniform), number of tori, then as
    ``_primitive_union``.  The torus segment counts and the sphere subdivision
    are chosen deterministically from the target.
    """
    rng = np.random.default_rng(seed)
    target = float(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi))))
    n_tori = int(rng.integers(1, 4))
    # Sphere: the largest subdivision whose 20*4^s triangles stay under a fifth of the target.
    s = 1
    while 20 * 4 ** (s + 1) <= target / 5 and s < 5:
        s += 1
    per_torus = max(64.0, (target - 20 * 4 ** s) / n_tori)
    n_minor = max(4, int(round(np.sqrt(per_torus / 2 / 1.6))))
    n_major = max(8, int(round(per_torus / 2 / n_minor)))
    return _primitive_union(rng, n_tori, (n_major, n_minor), s, 0.002)


def tri_soup(v, f):
    """Structure-of-arrays float32 triangle buffer ``[9][M]``: rows v0xyz, v1xyz, v2xyz."""
    t = v[f]                                  # [M, 3 corners, 3 coords]
    return np.ascontiguousarray(t.reshape(len(f), 9).T.astype(np.float32))
