"""UDF oracle: the unsigned distance field recovered from a directional one (Sec. III-A, Eq. 5),
float64.

Test infrastructure only (see the package docstring).

UDF(x) = min over directions theta of phi(x, theta), with phi infinite where the ray from x
misses.  Over a finite direction set {theta_j} this is a plain minimum; a point every
direction of which misses gets +inf.  The argument of the minimum is the lowest direction
index reaching it.
"""
import numpy as np

from oracle import geometry, mlp


def query_grid(points, dirs):
    """The (point, direction) grid as network inputs [5, n_points * n_dirs], point-major:
    query p * n_dirs + j = (x_p, theta_j, phi_j), angles of the unit directions by Eq. 1."""
    x = np.asarray(points, dtype=np.float64)
    theta, phi = geometry.angles_from_dirs(dirs)
    npt, nd = x.shape[1], theta.size
    return np.concatenate([np.repeat(x, nd, axis=1), np.tile(theta, npt)[None], np.tile(phi, npt)[None]])


def udf(field, points, dirs):
    """Eq. 5 over a direction set: ``field(rays5) -> (hit [N] bool, dist [N])``.

    Returns (udf [n_points], argmin [n_points], -1 where every direction misses).
    Pinned by the analytic sphere field (``||x| - r|`` when the set holds the direction to
    the nearest surface point) in the tests.
    """
    npt, nd = np.asarray(points).shape[1], np.asarray(dirs).shape[1]
    hit, dist = field(query_grid(points, dirs))
    D = np.where(hit, dist, np.inf).reshape(npt, nd)
    u = D.min(axis=1) if nd else np.full(npt, np.inf)
    arg = np.where(np.isfinite(u), D.argmin(axis=1) if nd else -1, -1)
    return u, arg


def network_field(params, width, depth, precision="fp64"):
    """The network as a field: a hit where logit > 0, phi = the distance output.  ``precision``
    "bf16" evaluates it through the emulated bfloat16 forward."""
    fwd = mlp.forward_bf16 if precision == "bf16" else mlp.forward

    def field(rays):
        logit, dist = fwd(params, width, depth, rays)
        return logit > 0.0, dist
    return field
