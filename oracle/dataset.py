"""Dataset oracle: the informative training-data sampler of Sec. V-B (Eqs. 8-12), float64.

Test infrastructure only (see the package docstring).

The sampler, in the paper's order:

1. Face points S_fc (Eq. 8): for each face (p0, p1, p2), ``s_fc`` points
   (1 - a - b) p0 + a p1 + b p2 from uniforms a, b.  Reading: a pair with
   a + b > 1 lies outside the face, so it is folded to (1 - a, 1 - b), which keeps
   the points uniform over the triangle.
2. Directions S_dr (Eq. 9): for each face, ``s_dr`` directions with polar angle
   theta0 = a pi and azimuth theta1 = 2 b pi (Eq. 1's parametrisation, polar from
   +z).  Reading: one set per face, shared by that face's points; every
   (point, direction) pair of a face is a candidate ray.
3. Rejection (the red and grey rays of Fig. 2a): the ray leaving the face point p
   along theta is dropped when it meets any triangle beyond ``eps`` (the offset
   that steps over p's own face), or when p is not inside the domain cube.  On a
   closed mesh a ray that enters the solid must leave it through another face, so
   this one test also drops the rays the odd-even rule marks as going inside.
4. Marching (Eq. 10): t_k = k t_exit / s_p for k = 1..s_p, where t_exit is where
   the ray leaves the domain cube [-1, 1]^3 (reading: the step spacing is not
   given).  At q = p + t_k theta the field looking back along -theta is t_k.
5. Infinite samples (Eqs. 11-12, Fig. 2b): looking on along theta from q the field
   is infinite (the ray was kept because it meets nothing); at theta +- pi/2 it is
   infinite and sampled only when that ray meets no triangle.  Reading: the
   +-pi/2 is applied to the polar angle, which gives the two opposite directions
   perpendicular to theta in its meridian plane,
   d+ = (cos theta0 cos theta1, cos theta0 sin theta1, -sin theta0), d- = -d+.

Samples come out in a fixed order: kept pairs by pair index (face, point,
direction), then k, then the kinds (back, forward, polar + pi/2, polar - pi/2).
Each sample is a network input (q, theta, phi) in the canonical ranges
theta in [0, pi], phi in [0, 2 pi), and a label t (+inf for "no hit").
"""
import numpy as np

from oracle import geometry

PI = np.pi
TWO_PI = 2.0 * np.pi


def face_points(tris, face_uv, s_fc, face_first=0, n_faces=None):
    """Eq. 8 points of faces ``face_first .. face_first + n_faces - 1``: [3, n_faces * s_fc].

    ``face_uv`` [2, m * s_fc] holds (a, b) of point j of face f at column f * s_fc + j.
    Reading: (a, b) with a + b > 1 is folded to (1 - a, 1 - b).
    Pinned: the points lie on their triangles, and the fold is uniform (tests).
    """
    v0, v1, v2 = geometry.triangles_from_soup(tris)
    m = v0.shape[1]
    n_faces = m - face_first if n_faces is None else n_faces
    faces = np.repeat(np.arange(face_first, face_first + n_faces), s_fc)
    cols = (faces * s_fc + np.tile(np.arange(s_fc), n_faces)).astype(np.int64)
    uv = np.asarray(face_uv, dtype=np.float64)
    a, b = uv[0, cols], uv[1, cols]
    fold = a + b > 1.0
    a = np.where(fold, 1.0 - a, a)
    b = np.where(fold, 1.0 - b, b)
    return (1.0 - a - b) * v0[:, faces] + a * v1[:, faces] + b * v2[:, faces]


def direction_angles(dir_uv):
    """Eq. 9: polar angle a pi and azimuth 2 b pi from uniforms ``dir_uv`` [2, K]."""
    uv = np.asarray(dir_uv, dtype=np.float64)
    return uv[0] * PI, uv[1] * TWO_PI


def cube_exit(o, d, half=1.0):
    """Distance along d at which a ray from a point o inside the cube [-half, half]^3 leaves it."""
    _, t_out, _ = geometry.cube_entry(o, d, half)
    return t_out


def _wrap_azimuth(phi):
    phi = np.where(phi >= TWO_PI, phi - TWO_PI, phi)
    return np.where(phi < 0.0, phi + TWO_PI, phi)


def sample_angles(theta0, theta1, kind):
    """Canonical (theta, phi) of sample ``kind`` for a kept ray of angles (theta0, theta1).

    kind 0: the reversed direction -theta (polar pi - theta0, azimuth + pi);
    kind 1: theta itself; kinds 2 and 3: polar theta0 + pi/2 and theta0 - pi/2,
    folded back into [0, pi] (a polar angle beyond a pole is the mirrored polar
    angle at the opposite azimuth).
    """
    theta0 = np.asarray(theta0, dtype=np.float64)
    theta1 = _wrap_azimuth(np.asarray(theta1, dtype=np.float64))
    if kind == 0:
        return PI - theta0, _wrap_azimuth(theta1 + PI)
    if kind == 1:
        return theta0, theta1
    t = theta0 + (0.5 * PI if kind == 2 else -0.5 * PI)
    over = t > PI
    under = t < 0.0
    flip = over | under
    t = np.where(over, TWO_PI - t, np.where(under, -t, t))
    return t, np.where(flip, _wrap_azimuth(theta1 + PI), theta1)


def sample_dataset(tris, face_uv, dir_uv, s_fc, s_dr, s_p, eps, face_first=0, n_faces=None, amb_tol=1e-6):
    """The sampler of Sec. V-B over faces ``face_first .. face_first + n_faces - 1``.

    ``tris`` [9, m] float32 corners (every triangle is intersected); ``face_uv``
    [2, m * s_fc]; ``dir_uv`` [2, m * s_dr] (direction j of face f at column
    f * s_dr + j).  Pair index i = (f - face_first) * s_fc * s_dr + point * s_dr + dir.

    Returns a dict: ``rays`` [5, N] (q, theta, phi), ``t`` [N], ``pair`` [N]
    (the pair index of each sample), ``kind`` [N], ``keep`` [P], ``fwd_ambiguous``
    [P] (the kept / dropped decision is not decided by the geometry: see
    ``geometry.nearest_hit``), ``perp_free`` [P, s_p, 2] and ``perp_ambiguous``
    [P, s_p, 2] (False where the pair is dropped), and the per-pair ``origin``,
    ``theta0``, ``theta1``, ``t_exit``.  ``amb_tol`` is passed to the ambiguity test of
    ``geometry.nearest_hit``.
    """
    v0, _, _ = geometry.triangles_from_soup(tris)
    m = v0.shape[1]
    n_faces = m - face_first if n_faces is None else n_faces
    P = n_faces * s_fc * s_dr
    pts = face_points(tris, face_uv, s_fc, face_first, n_faces)            # [3, n_faces * s_fc]
    th0_all, th1_all = direction_angles(dir_uv)
    pair = np.arange(P)
    f_local = pair // (s_fc * s_dr)
    point = (pair // s_dr) % s_fc
    dcol = (face_first + f_local) * s_dr + pair % s_dr
    o = pts[:, f_local * s_fc + point]
    th0, th1 = th0_all[dcol], th1_all[dcol]
    d = geometry.dirs_from_angles(th0, th1)
    inside = np.all(np.abs(o) < 1.0, axis=0)
    t_exit = np.where(inside, cube_exit(o, d), 0.0)
    fwd = geometry.nearest_hit(o, d, tris, t_min=eps, amb_tol=amb_tol)
    keep = (fwd["tri"] < 0) & (t_exit > 0.0)
    fwd_amb = fwd["ambiguous"]

    kept = np.flatnonzero(keep)
    k = np.arange(1, s_p + 1, dtype=np.float64)
    t_k = t_exit[kept][:, None] * k[None, :] / s_p                           # [A, s_p]
    q = o[:, kept][:, :, None] + d[:, kept][:, :, None] * t_k[None]           # [3, A, s_p]
    st0, ct0 = np.sin(th0[kept]), np.cos(th0[kept])
    dp = np.stack([ct0 * np.cos(th1[kept]), ct0 * np.sin(th1[kept]), -st0])  # [3, A] (polar + pi/2)
    qf = q.reshape(3, -1)
    dpf = np.repeat(dp, s_p, axis=1)
    perp_free = np.zeros((P, s_p, 2), dtype=bool)
    perp_amb = np.zeros((P, s_p, 2), dtype=bool)
    for s, sign in enumerate((1.0, -1.0)):
        h = geometry.nearest_hit(qf, sign * dpf, tris, t_min=0.0, amb_tol=amb_tol)
        perp_free[kept, :, s] = (h["tri"] < 0).reshape(len(kept), s_p)
        perp_amb[kept, :, s] = h["ambiguous"].reshape(len(kept), s_p)

    rays, ts, src, kinds = [], [], [], []
    for a, i in enumerate(kept):
        for j in range(s_p):
            for kind in range(4):
                if kind >= 2 and not perp_free[i, j, kind - 2]:
                    continue
                theta, phi = sample_angles(th0[i], th1[i], kind)
                rays.append([q[0, a, j], q[1, a, j], q[2, a, j], float(theta), float(phi)])
                ts.append(t_k[a, j] if kind == 0 else np.inf)
                src.append(i)
                kinds.append(kind)
    rays = np.array(rays, dtype=np.float64).reshape(-1, 5).T
    return {"rays": rays, "t": np.array(ts, dtype=np.float64), "pair": np.array(src, dtype=np.int64),
            "kind": np.array(kinds, dtype=np.int64), "keep": keep, "fwd_ambiguous": fwd_amb,
            "perp_free": perp_free, "perp_ambiguous": perp_amb, "origin": o, "theta0": th0, "theta1": th1,
            "t_exit": t_exit}
