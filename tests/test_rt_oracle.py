"""Pins of the ray tracer's CPU oracle against closed forms and invariants
(CPU only).  The oracle's per-pixel result is what the queue-driven tracer of
Section V-B must reproduce bit for bit."""
import math

import numpy as np
import pytest

from oracle import raytrace as rt
from workloads import scenes

F = np.float32


def _scene(spheres=(), planes=(), light=(0.0, 1.0, 0.0), shade=(0.25, 0.75),
           background=(0.5, 0.25, 0.125), max_bounces=2):
    return dict(spheres=np.array(spheres, dtype=F).reshape(-1, 10),
                planes=np.array(planes, dtype=F).reshape(-1, 8),
                camera=np.zeros(7, F), light=np.array(light, F), shade=np.array(shade, F),
                background=np.array(background, F), max_bounces=max_bounces)


def _sph(cx, cy, cz, r, alb=(1.0, 1.0, 1.0), refl=0.0):
    return [cx, cy, cz, F(r) * F(r), F(1) / F(r), *alb, refl, 0.0]


def _rays(o, d):
    o = np.array(o, F).reshape(-1, 3)
    d = np.array(d, F).reshape(-1, 3)
    return [o[:, i].copy() for i in range(3)], [d[:, i].copy() for i in range(3)]


def test_sphere_distance_closed_form():
    """Ray along -z from the origin to a unit sphere at z = -5: t = 4; from
    inside the sphere (origin at its centre): t = r."""
    sc = _scene(spheres=[_sph(0, 0, -5, 1)])
    o, d = _rays([[0, 0, 0], [0, 0, -5]], [[0, 0, -1], [0, 0, -1]])
    hit, t = rt.nearest_hit(sc, o, d)
    assert hit.tolist() == [0, 0]
    assert t.tolist() == [4.0, 1.0]


def test_sphere_miss_and_tangent_side():
    """A ray passing at distance 1.5 from a unit sphere misses it."""
    sc = _scene(spheres=[_sph(0, 0, -5, 1)])
    o, d = _rays([[1.5, 0, 0]], [[0, 0, -1]])
    hit, t = rt.nearest_hit(sc, o, d)
    assert hit.tolist() == [-1] and math.isinf(float(t[0]))


def test_plane_distance_and_facing():
    """Plane y = 0 facing +y: from height 2 straight down t = 2; a ray going
    up, or parallel to the plane, does not hit it (back faces and den = 0)."""
    sc = _scene(planes=[[0, 1, 0, 0, 1, 1, 1, 0]])
    o, d = _rays([[0, 2, 0], [0, 2, 0], [0, 2, 0]], [[0, -1, 0], [0, 1, 0], [1, 0, 0]])
    hit, t = rt.nearest_hit(sc, o, d)
    assert hit.tolist() == [0, -1, -1]
    assert float(t[0]) == 2.0


def test_nearest_wins_regardless_of_index_and_tie_goes_to_first():
    far, near = _sph(0, 0, -10, 1), _sph(0, 0, -5, 1)
    o, d = _rays([[0, 0, 0]], [[0, 0, -1]])
    assert rt.nearest_hit(_scene(spheres=[far, near]), o, d)[0].tolist() == [1]
    assert rt.nearest_hit(_scene(spheres=[near, far]), o, d)[0].tolist() == [0]
    assert rt.nearest_hit(_scene(spheres=[near, near]), o, d)[0].tolist() == [0]
    # a sphere in front of the plane hides it; spheres come first on equal t
    sc = _scene(spheres=[_sph(0, 1, 0, 1)], planes=[[0, 1, 0, 0, 1, 1, 1, 0]])
    o, d = _rays([[0, 5, 0]], [[0, -1, 0]])
    hit, t = rt.nearest_hit(sc, o, d)
    assert hit.tolist() == [0] and float(t[0]) == 3.0


def test_diffuse_hit_colour_closed_form():
    """Straight down onto a plane lit from straight above: n.L = 1, so the
    colour is albedo * (ambient + diffuse) and the path ends (refl 0)."""
    sc = _scene(planes=[[0, 1, 0, 0, 0.5, 0.25, 1.0, 0.0]])
    o, d = _rays([[0, 3, 0]], [[0, -1, 0]])
    img, segs = rt.trace(sc, o, d)
    assert segs.tolist() == [1]
    assert img[0].tolist() == [0.5, 0.25, 1.0]  # ambient + diffuse = 1 exactly


def test_mirror_bounce_closed_form():
    """A vertical ray on a plane of reflectivity 1/2 reflects straight up and
    escapes: colour = albedo * 1 + 1/2 * background; two segments."""
    sc = _scene(planes=[[0, 1, 0, 0, 0.5, 0.5, 0.5, 0.5]])
    o, d = _rays([[0, 3, 0]], [[0, -1, 0]])
    img, segs = rt.trace(sc, o, d)
    assert segs.tolist() == [2]
    assert img[0].tolist() == [0.75, 0.625, 0.5625]


def test_light_from_behind_gives_ambient_only():
    sc = _scene(planes=[[0, 1, 0, 0, 1.0, 1.0, 1.0, 0.0]], light=(0.0, -1.0, 0.0))
    o, d = _rays([[0, 3, 0]], [[0, -1, 0]])
    img, _ = rt.trace(sc, o, d)
    assert img[0].tolist() == [0.25, 0.25, 0.25]


def test_bounce_limit_between_parallel_mirrors():
    """Two facing mirrors y = 0 and y = 4: a vertical ray bounces until the
    bounce limit; colour is a geometric series of albedo * shade."""
    for mb in (0, 1, 2, 4):
        sc = _scene(planes=[[0, 1, 0, 0, 1, 1, 1, 0.5], [0, -1, 0, -4, 1, 1, 1, 0.5]],
                    light=(0.0, 1.0, 0.0), shade=(1.0, 0.0), max_bounces=mb)
        o, d = _rays([[0, 2, 0]], [[0, -1, 0]])
        img, segs = rt.trace(sc, o, d)
        assert segs.tolist() == [mb + 1]
        expect = sum(0.5 ** i for i in range(mb + 1))
        assert img[0, 0] == F(expect)


def test_empty_scene_is_background():
    sc = scenes.cornell_scene(32, 24)
    sc = dict(sc, spheres=np.zeros((0, 10), F), planes=np.zeros((0, 8), F))
    img, segs = rt.render(sc, 32, 24)
    assert (segs == 1).all()
    assert (img == sc["background"][None, :]).all()


def test_primary_rays_are_unit_and_centred():
    sc = scenes.complex_scene(20260601, 64, 48)
    o, d = rt.primary_rays(sc, 64, 48)
    n2 = (d[0].astype(np.float64) ** 2 + d[1] ** 2 + d[2] ** 2)
    assert np.abs(n2 - 1).max() < 1e-6
    assert (d[2] < 0).all()
    # columns 31 and 32 straddle the image centre: x components of opposite sign
    w = 64
    assert (d[0][31::w] < 0).all() and (d[0][32::w] > 0).all()


@pytest.mark.parametrize("name", ["complex", "cornell"])
def test_scene_renders_invariants(name):
    W, H = 48, 32
    sc = scenes.complex_scene(20260601, W, H) if name == "complex" else scenes.cornell_scene(W, H)
    img, segs = rt.render(sc, W, H)
    assert img.shape == (W * H, 3) and img.dtype == np.float32
    assert (segs >= 1).all() and (segs <= sc["max_bounces"] + 1).all()
    assert np.isfinite(img).all() and (img >= 0).all()
    # pixels rendered one by one give the same bits as the whole image
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    sel = np.arange(0, W * H, 37)
    img2, segs2 = rt.render(sc, W, H, xs.ravel()[sel], ys.ravel()[sel])
    assert np.array_equal(img2.view(np.uint32), img[sel].view(np.uint32))
    assert np.array_equal(segs2, segs[sel])
