"""Scene descriptions for the render workloads (camera, light, material, sizes).

The paper gives no camera, light or material values; these are the readings
used throughout (pinhole camera, Z-up as in the paper's figures, one point
light, grey Lambertian albedo, black background):

* small / full render: eye (0, -3, 0.5) looking at the origin, vertical field
  of view 40 degrees, point light at (2, -2, 3) with intensity 10 per channel,
  albedo 0.7;
* multi-object render: eye (0, -12, 6), vertical field of view 50 degrees, light
  at (4, -6, 10) with intensity 120, instances on a 4 x 4 grid in the z = 0 plane.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class Camera:
    eye: tuple = (0.0, -3.0, 0.5)
    target: tuple = (0.0, 0.0, 0.0)
    up: tuple = (0.0, 0.0, 1.0)
    vfov_deg: float = 40.0


@dataclass
class Light:
    position: tuple = (2.0, -2.0, 3.0)
    intensity: tuple = (10.0, 10.0, 10.0)


@dataclass
class RenderConfig:
    width: int = 64
    height: int = 64
    spp: int = 1
    bounces: int = 3
    rr_start: int = 3          # Russian roulette after the scatter of bounce index >= rr_start
    seed: int = 0
    eps: float = 1e-3          # offset of secondary-ray origins along the normal
    albedo: tuple = (0.7, 0.7, 0.7)
    camera: Camera = field(default_factory=Camera)
    light: Light = field(default_factory=Light)


def small_render():
    """64 x 64, 1 sample per pixel, 3 bounces (no Russian roulette reached)."""
    return RenderConfig(64, 64, 1, 3, 3, 0)


def full_render(spp=64):
    """1920 x 1080, 64 samples per pixel, 4 bounces, Russian roulette after bounce 2."""
    return RenderConfig(1920, 1080, spp, 4, 2, 0)


def multi_object_render(spp=16):
    """1280 x 720, 16 samples per pixel, 3 bounces, camera pulled back to see 16 instances."""
    return RenderConfig(1280, 720, spp, 3, 2, 0, camera=Camera(eye=(0.0, -12.0, 6.0), vfov_deg=50.0),
                        light=Light(position=(4.0, -6.0, 10.0), intensity=(120.0, 120.0, 120.0)))


def _rotation_from_quaternion(q):
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def instance_layout(n_instances=16, n_networks=8, seed=10, spacing=3.6, jitter=0.1):
    """Rigid instances on a jittered square grid in the z = 0 plane.

    Instance i uses network ``i mod n_networks``, a uniform random rotation (from a
    normalised Gaussian quaternion) and the translation of grid cell i plus
    U(-jitter, jitter) per axis.  Every object lies in [-0.97, 0.97]^3, so its
    vertices are within 1.68 of its centre, and ``spacing - 2 jitter > 3.36``
    keeps the instances disjoint.  Returns dicts with ``R`` (3x3, object to world),
    ``T`` (3) and ``net``.
    """
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(n_instances)))
    out = []
    for i in range(n_instances):
        g = rng.normal(size=4)
        R = _rotation_from_quaternion(g / np.linalg.norm(g))
        gx, gy = i % side, i // side
        base = np.array([(gx - (side - 1) / 2) * spacing, (gy - (side - 1) / 2) * spacing, 0.0])
        T = base + rng.uniform(-jitter, jitter, size=3)
        out.append({"R": R, "T": T, "net": i % n_networks})
    return out
