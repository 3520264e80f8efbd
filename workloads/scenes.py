"""Seeded synthetic scenes for the tile-based wavefront ray tracer.

These are the two scenes of the paper's ray-tracing workload (Section V-B,
tile-based wavefront ray tracing): a complex scene of 100 spheres on a ground
plane with two-bounce reflections, and a Cornell-box-like scene of two spheres,
a floor and three walls with four reflections.  The paper names the scenes
only; their geometry, materials, camera and light here are our own choice.

Only data is defined here (no tracing arithmetic).  A scene is a dict:
  spheres  float32 [S, 10]: cx cy cz r2 inv_r albedo_r albedo_g albedo_b refl 0
           (r2 = r*r and inv_r = 1/r rounded to float32 here, once)
  planes   float32 [P, 8]:  nx ny nz d albedo_r albedo_g albedo_b refl
           (the plane n.p = d with unit axis-aligned normal n, facing the scene)
  camera   float32 [7]: eye_x eye_y eye_z sx sy ax ay -- the primary ray of
           pixel (x, y) has direction ((x + 0.5) sx - ax, ay - (y + 0.5) sy, -1)
           before normalisation
  light    float32 [3]: unit vector towards a directional light
  shade    float32 [2]: ambient, diffuse (shade = ambient + diffuse * max(0, n.L))
  background float32 [3]
  max_bounces int
"""
from __future__ import annotations

import math

import numpy as np

from . import splitmix64

F = np.float32


def _unit(seed: int, stream: int, k: int) -> float:
    """Uniform in [0, 1) from the counter-based stream (53-bit mantissa)."""
    return (splitmix64(seed, (stream << 32) | k) >> 11) / float(1 << 53)


def _camera(eye, width: int, height: int, fov_deg: float, tilt: float):
    th = math.tan(math.radians(fov_deg) / 2.0)
    aspect = width / height
    return np.array([eye[0], eye[1], eye[2], 2.0 * th * aspect / width, 2.0 * th / height,
                     th * aspect, th + tilt], dtype=F)


def _light(x, y, z):
    n = math.sqrt(x * x + y * y + z * z)
    return np.array([x / n, y / n, z / n], dtype=F)


def _sphere(cx, cy, cz, r, alb, refl):
    return [cx, cy, cz, F(r) * F(r), F(1.0) / F(r), alb[0], alb[1], alb[2], refl, 0.0]


def complex_scene(seed: int, width: int, height: int) -> dict:
    """100 spheres (radius 0.25-0.45) resting on the plane y = 0 on a jittered
    10 x 10 grid; every other sphere is a mirror (reflectivity 0.7), the plane
    reflects 0.3; at most two bounces."""
    sph = []
    for i in range(100):
        gx, gz = i % 10, i // 10
        r = 0.25 + 0.2 * _unit(seed, 1, 4 * i)
        cx = -4.5 + gx + 0.3 * (_unit(seed, 1, 4 * i + 1) - 0.5)
        cz = -4.0 - gz - 0.3 * (_unit(seed, 1, 4 * i + 2) - 0.5)
        alb = [0.2 + 0.8 * _unit(seed, 2, 3 * i + c) for c in range(3)]
        sph.append(_sphere(cx, r, cz, r, alb, 0.7 if i % 2 == 0 else 0.0))
    planes = [[0.0, 1.0, 0.0, 0.0, 0.6, 0.6, 0.6, 0.3]]
    return dict(name="complex", spheres=np.array(sph, dtype=F), planes=np.array(planes, dtype=F),
                camera=_camera((0.0, 2.5, 2.0), width, height, 60.0, -0.35),
                light=_light(0.3, 1.0, 0.5), shade=np.array([0.15, 0.85], dtype=F),
                background=np.array([0.55, 0.7, 0.9], dtype=F), max_bounces=2)


def cornell_scene(width: int, height: int) -> dict:
    """Two mirror spheres (reflectivity 0.9) on a floor (0.4) between a red
    left wall, a green right wall and a white back wall (0.5, 0.5, 0.6); at
    most four bounces."""
    sph = [_sphere(-0.6, 0.5, -3.5, 0.5, (0.9, 0.9, 0.9), 0.9),
           _sphere(0.7, 0.7, -2.8, 0.7, (0.95, 0.85, 0.6), 0.9)]
    planes = [[0.0, 1.0, 0.0, 0.0, 0.8, 0.8, 0.8, 0.4],     # floor y = 0
              [1.0, 0.0, 0.0, -1.5, 0.8, 0.15, 0.15, 0.5],  # left wall x = -1.5
              [-1.0, 0.0, 0.0, -1.5, 0.15, 0.8, 0.15, 0.5],  # right wall x = 1.5
              [0.0, 0.0, 1.0, -5.0, 0.85, 0.85, 0.85, 0.6]]  # back wall z = -5
    return dict(name="cornell", spheres=np.array(sph, dtype=F), planes=np.array(planes, dtype=F),
                camera=_camera((0.0, 1.2, 1.5), width, height, 55.0, -0.15),
                light=_light(-0.2, 1.0, 0.6), shade=np.array([0.2, 0.8], dtype=F),
                background=np.array([0.05, 0.05, 0.08], dtype=F), max_bounces=4)
