"""Multi-object oracle: several networks placed as rigid instances (test infrastructure only).

Scenes made of many objects are the paper's stated future work (Sec. VII); the reading used
here: instance i maps object space to world space by x_world = R_i x_object + T_i; a world
ray is moved into each instance's object space (o' = R^T (o - T), d' = R^T d), queried from
the entry of that object's cube [-1,1]^3 like a single network, and the nearest hit over all
instances wins (rigid maps preserve distances; a hit needs logit > 0 and a distance >= 0;
ties go to the lower instance index).  The shading normal uses the world-space gradient
R g_object.  A shadow ray is blocked when any instance reports a hit before the light.
Pinned by invariants in the tests: one instance with the identity transform renders exactly
as the single-network scene, and moving the whole scene, camera and light by one rigid map
leaves the image unchanged.
"""
import numpy as np

from . import geometry, mlp


class MultiScene:
    def __init__(self, nets, instances, logit_margin=1e-4, precision="fp64"):
        """nets: list of (params, width, depth); instances: dicts with R (3x3), T (3), net.
        precision "bf16": networks evaluated as ``mlp.forward_bf16`` / ``mlp.backward_input_bf16``."""
        self.nets = nets
        self.inst = [(np.asarray(d["R"], np.float64), np.asarray(d["T"], np.float64), int(d["net"])) for d in instances]
        self.margin = logit_margin
        self.bf16 = precision == "bf16"

    def _query_all(self, o, d, want_grad):
        n = o.shape[1]
        out = []
        for R, T, k in self.inst:
            p, w, depth = self.nets[k]
            oo = R.T @ (o - T[:, None])
            dd = R.T @ d
            t_in, t_out, inbox = geometry.cube_entry(oo, dd)
            t0 = np.maximum(t_in, 0.0)
            q = oo + t0[None] * dd
            th, ph = geometry.angles_from_dirs(dd)
            rays = np.concatenate([q, th[None], ph[None]])
            logit, dist = (mlp.forward_bf16 if self.bf16 else mlp.forward)(p, w, depth, rays)
            t = t0 + dist
            hit = inbox & (logit > 0.0) & (t >= 0.0)
            robust = ~inbox | ((np.abs(logit) > self.margin) & (np.abs(t) > self.margin))
            g = None
            if want_grad:
                if self.bf16:
                    gr = mlp.backward_input_bf16(p, w, depth, rays, np.zeros(n), np.ones(n))
                else:
                    gr, _ = mlp.backward(p, w, depth, rays, np.zeros(n), np.ones(n))
                g = R @ gr[0:3]
            out.append((hit, t, g, robust))
        return out

    def intersect(self, o, d, t_max):
        res = self._query_all(o, d, True)
        n = o.shape[1]
        best_t = np.full(n, np.inf)
        best_g = np.zeros((3, n))
        robust = np.ones(n, dtype=bool)
        for hit, t, g, rb in res:
            robust &= rb
            closer = hit & (t < best_t)
            best_t = np.where(closer, t, best_t)
            best_g = np.where(closer[None], g, best_g)
        # two instances at nearly the same distance leave the winner undecided
        for hit, t, _, _ in res:
            robust &= ~(hit & (t != best_t) & (np.abs(t - best_t) <= self.margin * (1.0 + np.abs(best_t))))
        hit_any = np.isfinite(best_t)
        gn = np.linalg.norm(best_g, axis=0)
        robust &= ~(hit_any & (gn < self.margin * 10.0))
        return hit_any, best_t, best_g, robust

    def occluded(self, o, d, t_max):
        res = self._query_all(o, d, False)
        occ = np.zeros(o.shape[1], dtype=bool)
        robust = np.ones(o.shape[1], dtype=bool)
        for hit, t, _, rb in res:
            occ |= hit & (t < t_max)
            robust &= rb & ~(hit & (np.abs(t - t_max) <= self.margin * (1.0 + np.abs(t_max))))
        return occ, robust
