"""Geometry oracle: angles, cube entry and brute-force nearest hit, float64.

Test infrastructure only (see the package docstring).
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def dirs_from_angles(theta, phi):
    """Unit direction of polar angle ``theta`` (from +z) and azimuth ``phi`` (Sec. III-A, Eq. 1).

    d = (cos(phi) sin(theta), sin(phi) sin(theta), cos(theta)).  Eq. 1 names the
    azimuth theta_0 and the polar angle theta_1; this uses theta = polar,
    phi = azimuth.  Pinned by closed forms (poles, equator) in the tests.
    """
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    st = np.sin(theta)
    return np.stack([np.cos(phi) * st, np.sin(phi) * st, np.cos(theta)], axis=0)


def angles_from_dirs(d):
    """Inverse of Eq. 1 for a direction ``d`` [3, N] (any positive length).

    theta = angle between d and +z in [0, pi]; phi = atan2(dy, dx) wrapped into
    [0, 2 pi); phi = 0 on the z axis.  Pinned by round trip and closed forms.
    """
    d = np.asarray(d, dtype=np.float64)
    theta = np.arctan2(np.hypot(d[0], d[1]), d[2])
    phi = np.arctan2(d[1], d[0])
    phi = np.where(phi < 0.0, phi + TWO_PI, phi)
    phi = np.where(phi >= TWO_PI, phi - TWO_PI, phi)
    return theta, phi


def cube_entry(o, d, half=1.0):
    """Slab test of rays against the domain cube [-half, half]^3.

    Returns ``(t_in, t_out, hit)``; ``hit`` is False when the ray misses the cube
    or the cube lies behind the origin.  A query point outside the cube is moved
    to ``o + max(t_in, 0) d`` before the network is evaluated (the field is only
    defined on the bounded box B, Sec. III-A).  Pinned by axis-aligned closed forms.
    """
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (-half - o) * inv
        t1 = (half - o) * inv
    lo = np.minimum(t0, t1)
    hi = np.maximum(t0, t1)
    # A zero direction component: the ray is inside the slab for all t or for none.
    inside = (o >= -half) & (o <= half)
    lo = np.where(d == 0.0, np.where(inside, -np.inf, np.inf), lo)
    hi = np.where(d == 0.0, np.where(inside, np.inf, -np.inf), hi)
    t_in = lo.max(axis=0)
    t_out = hi.min(axis=0)
    hit = (t_in <= t_out) & (t_out > 0.0)
    return t_in, t_out, hit


def triangles_from_soup(tris):
    """Split the ``[9][M]`` float32 soup into float64 corner arrays ``v0, v1, v2`` of shape [3, M]."""
    t = np.asarray(tris, dtype=np.float64)
    return t[0:3], t[3:6], t[6:9]


def nearest_hit(orig, dirs, tris, t_min=0.0, t_max=np.inf, amb_tol=1e-6):
    """Nearest ray/triangle hit by linear search over every triangle.

    The paper's baseline search for the nearest triangle along a ray (Sec. I)
    and its ray shooting for labels (Sec. VI-B), with the Moller-Trumbore
    (1997) two-sided test: for edges e1 = v1 - v0, e2 = v2 - v0,
    p = d x e2, det = e1 . p (det == 0 is a miss), s = o - v0,
    u = s . p / det, q = s x e1, v = d . q / det, t = e2 . q / det; accepted
    when u >= 0, v >= 0, u + v <= 1 (edges inclusive) and t_min < t < t_max.
    The nearest accepted t wins; exact ties go to the lowest triangle index.
    ``crossings`` counts every accepted hit (the odd-even rule of Sec. V-B: an
    odd count means the origin is inside a closed mesh).

    Also returns, per ray, ``ambiguous`` (some triangle's hit point lies within
    ``amb_tol`` of its boundary in barycentric units, the ray is within
    ``amb_tol`` of grazing a plane it may hit, or a hit lies within ``amb_tol``
    of t_min) and ``t_second`` (second-nearest accepted t), so that parity
    checks can exclude rays whose answer is not decided by the geometry.

    Pinned by the quad and single-triangle closed forms, the icosphere sandwich
    bounds and an exact rational brute force on tiny meshes.
    """
    o = np.asarray(orig, dtype=np.float64)
    d = np.asarray(dirs, dtype=np.float64)
    v0, v1, v2 = triangles_from_soup(tris)
    n = o.shape[1]
    best_t = np.full(n, np.inf)
    second_t = np.full(n, np.inf)
    best_i = np.full(n, -1, dtype=np.int64)
    crossings = np.zeros(n, dtype=np.int64)
    ambiguous = np.zeros(n, dtype=bool)
    dlen = np.linalg.norm(d, axis=0)
    for i in range(v0.shape[1]):
        e1 = (v1[:, i] - v0[:, i])[:, None]
        e2 = (v2[:, i] - v0[:, i])[:, None]
        p = np.cross(d, e2, axis=0)
        det = np.sum(e1 * p, axis=0)
        s = o - v0[:, i][:, None]
        q = np.cross(s, e1, axis=0)
        ok = det != 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            u = np.sum(s * p, axis=0) / det
            v = np.sum(d * q, axis=0) / det
            t = np.sum(e2 * q, axis=0) / det
            accept = ok & (u >= 0.0) & (v >= 0.0) & (u + v <= 1.0) & (t > t_min) & (t < t_max)
            margin = np.minimum(np.minimum(u, v), 1.0 - u - v)
        with np.errstate(invalid="ignore"):
            in_range = ok & (t > t_min - amb_tol) & (t < t_max + amb_tol)
            amb = in_range & (np.abs(margin) < amb_tol)
            amb |= ok & (np.abs(t - t_min) < amb_tol) & (margin > -amb_tol)
            area2 = np.linalg.norm(np.cross(e1, e2, axis=0))
            cosang = np.abs(det) / (area2 * dlen)
            amb |= (cosang < amb_tol) & ~(ok & (margin < -1e-3))
        ambiguous |= amb
        crossings += accept
        closer = accept & (t < best_t)
        second_t = np.where(accept & ~closer, np.minimum(second_t, t), second_t)
        second_t = np.where(closer, best_t, second_t)
        best_t = np.where(closer, t, best_t)
        best_i = np.where(closer, i, best_i)
    return {"t": best_t, "tri": best_i, "crossings": crossings, "ambiguous": ambiguous, "t_second": second_t}


def face_normals(tris):
    """Unit geometric normals (e1 x e2 normalised) of the soup's triangles, [3, M]."""
    v0, v1, v2 = triangles_from_soup(tris)
    n = np.cross(v1 - v0, v2 - v0, axis=0)
    return n / np.linalg.norm(n, axis=0, keepdims=True)
