"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *draws* inputs: procedural triangle meshes, ray origins and
unit directions, network parameters and scene descriptions.  It holds none of
the method's arithmetic (no ray/triangle test, no angle parametrisation, no
encoding, no network evaluation), so both sides of every parity check can
import it without sharing any computation.

All randomness uses NumPy's PCG64 through ``numpy.random.default_rng(seed)``;
the draw order of every generator is fixed and documented in its docstring.
"""
from .meshes import icosphere, torus, union, jitter_vertices, training_mesh, multi_object_mesh, tri_soup
from .rays import uniform_cube_rays, training_rays, render_rays, unit_ball_rays, area_weighted_surface_points, dataset_uniforms, grid_points
from .weights import layer_shapes, param_count, xavier_params, random_params, multi_object_network_shape, paper_params
from .scenes import Camera, Light, RenderConfig, small_render, full_render, multi_object_render, instance_layout

__all__ = [
    "icosphere", "torus", "union", "jitter_vertices", "training_mesh", "multi_object_mesh", "tri_soup",
    "uniform_cube_rays", "training_rays", "render_rays", "unit_ball_rays", "area_weighted_surface_points", "dataset_uniforms", "grid_points",
    "layer_shapes", "param_count", "xavier_params", "random_params", "multi_object_network_shape", "paper_params",
    "Camera", "Light", "RenderConfig", "small_render", "full_render", "multi_object_render", "instance_layout",
]
