"""CPU oracle of the wavefront ray tracer's image.  TEST INFRASTRUCTURE ONLY.

The queue-driven tracer of the paper's ray-tracing workload (Section V-B,
tile-based wavefront ray tracing) re-enqueues reflective bounces until every
path ends; what it computes per pixel does not depend on the queue, the tile
or the order in which paths are traced.  This module computes that per-pixel
result directly: every pixel's path, segment by segment, in float32 with each
operation rounded to float32 in the order written below (numpy float32
arithmetic, no fused multiply-add; division and square root correctly
rounded), so a kernel that evaluates the same expressions in the same order
produces the same bits.

Per segment from origin o along unit direction d:
  spheres (in index order): oc = o - c; b = oc.d; q = oc.oc - r2; disc = b*b - q;
      if disc >= 0: s = sqrt(disc); t = (-b) - s, and if t <= EPS then t = (-b) + s;
      a sphere is a candidate when t > EPS
  planes (after the spheres, in index order): den = n.d; if den < 0:
      t = (pd - n.o) / den, a candidate when t > EPS
  the nearest candidate wins; on equal t the earlier object (x.y + ... is
  evaluated as ((x0*y0) + (x1*y1)) + (x2*y2) everywhere)
  miss: colour += thr * background, the path ends
  hit at h = o + t*d with normal n (sphere: (h - c) * inv_r; plane: its n):
      lam = max(0, n.L); colour_c += (thr * albedo_c) * (ambient + diffuse * lam)
      if refl > 0 and depth < max_bounces: k = 2 * (d.n); d = d - k*n;
      o = h + BIAS*n; thr = thr * refl; depth += 1; next segment
      else the path ends
Primary ray of pixel (x, y): o = eye, d = normalise(((x + 0.5) sx - ax,
ay - (y + 0.5) sy, -1)) with normalise(v) = v * (1 / sqrt(v.v)).

Returns the image (float32 [H, W, 3]) and the number of segments traced per
pixel (uint32 [H, W]).
"""
from __future__ import annotations

import numpy as np

F = np.float32
EPS = F(1e-4)
BIAS = F(1e-3)


def _dot(ax, ay, az, bx, by, bz):
    return (ax * bx + ay * by) + az * bz


def primary_rays(scene: dict, width: int, height: int, xs=None, ys=None):
    """Origins and unit directions of the primary rays, float32."""
    cam = scene["camera"]
    if xs is None:
        ys, xs = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
        xs, ys = xs.ravel(), ys.ravel()
    fx = xs.astype(F) + F(0.5)
    fy = ys.astype(F) + F(0.5)
    dx = fx * cam[3] - cam[5]
    dy = cam[6] - fy * cam[4]
    dz = np.full_like(dx, F(-1.0))
    inv = F(1.0) / np.sqrt(_dot(dx, dy, dz, dx, dy, dz))
    n = len(dx)
    o = [np.full(n, cam[0], F), np.full(n, cam[1], F), np.full(n, cam[2], F)]
    return o, [dx * inv, dy * inv, dz * inv]


def nearest_hit(scene: dict, o, d):
    """Index of the nearest object (spheres first, then planes; -1 = miss)
    and its distance, per ray."""
    ox, oy, oz = o
    dx, dy, dz = d
    n = len(ox)
    best_t = np.full(n, np.inf, F)
    best = np.full(n, -1, np.int64)
    for i, s in enumerate(scene["spheres"]):
        cx, cy, cz, r2 = s[0], s[1], s[2], s[3]
        px, py, pz = ox - cx, oy - cy, oz - cz
        b = _dot(px, py, pz, dx, dy, dz)
        q = _dot(px, py, pz, px, py, pz) - r2
        disc = b * b - q
        ok = disc >= F(0)
        sq = np.sqrt(np.where(ok, disc, F(0)))
        t = (-b) - sq
        t = np.where(t <= EPS, (-b) + sq, t)
        take = ok & (t > EPS) & (t < best_t)
        best_t = np.where(take, t, best_t)
        best = np.where(take, i, best)
    ns = len(scene["spheres"])
    for j, p in enumerate(scene["planes"]):
        nx, ny, nz, pd = p[0], p[1], p[2], p[3]
        den = _dot(nx, ny, nz, dx, dy, dz)
        ok = den < F(0)
        t = (pd - _dot(nx, ny, nz, ox, oy, oz)) / np.where(ok, den, F(-1))
        take = ok & (t > EPS) & (t < best_t)
        best_t = np.where(take, t, best_t)
        best = np.where(take, ns + j, best)
    return best, best_t


def render(scene: dict, width: int, height: int, xs=None, ys=None):
    """Image (float32 [n, 3]) and segments per pixel (uint32 [n]) for the
    pixels (xs, ys), by default the whole image in row-major order."""
    o, d = primary_rays(scene, width, height, xs, ys)
    return trace(scene, o, d)


def trace(scene: dict, o, d):
    """Colour (float32 [n, 3]) and segments (uint32 [n]) of the paths that
    start at origins o and unit directions d (lists of three float32 arrays,
    overwritten)."""
    o = [np.array(c, dtype=F) for c in o]
    d = [np.array(c, dtype=F) for c in d]
    n = len(o[0])
    col = [np.zeros(n, F), np.zeros(n, F), np.zeros(n, F)]
    thr = np.ones(n, F)
    segs = np.zeros(n, np.uint32)
    alive = np.arange(n)
    sph, pl = scene["spheres"], scene["planes"]
    ns = len(sph)
    L = scene["light"]
    amb, dif = scene["shade"][0], scene["shade"][1]
    bg = scene["background"]
    for depth in range(scene["max_bounces"] + 1):
        if len(alive) == 0:
            break
        oa = [c[alive] for c in o]
        da = [c[alive] for c in d]
        ta = thr[alive]
        segs[alive] += np.uint32(1)
        hit, t = nearest_hit(scene, oa, da)
        miss = hit < 0
        for c in range(3):
            col[c][alive[miss]] = col[c][alive[miss]] + ta[miss] * bg[c]
        h_idx = np.nonzero(~miss)[0]
        if len(h_idx) == 0:
            break
        a = alive[h_idx]
        obj = hit[h_idx]
        th = t[h_idx]
        hx = oa[0][h_idx] + th * da[0][h_idx]
        hy = oa[1][h_idx] + th * da[1][h_idx]
        hz = oa[2][h_idx] + th * da[2][h_idx]
        is_s = obj < ns
        si = np.where(is_s, obj, 0)
        pi = np.where(is_s, 0, obj - ns)
        S = sph[si] if ns else np.zeros((len(obj), 10), F)
        P = pl[pi] if len(pl) else np.zeros((len(obj), 8), F)
        nx = np.where(is_s, (hx - S[:, 0]) * S[:, 4], P[:, 0])
        ny = np.where(is_s, (hy - S[:, 1]) * S[:, 4], P[:, 1])
        nz = np.where(is_s, (hz - S[:, 2]) * S[:, 4], P[:, 2])
        alb = [np.where(is_s, S[:, 5 + c], P[:, 4 + c]) for c in range(3)]
        refl = np.where(is_s, S[:, 8], P[:, 7])
        lam = _dot(nx, ny, nz, L[0], L[1], L[2])
        lam = np.where(lam < F(0), F(0), lam)
        shade = amb + dif * lam
        tt = ta[h_idx]
        for c in range(3):
            col[c][a] = col[c][a] + (tt * alb[c]) * shade
        go = (refl > F(0)) & (depth < scene["max_bounces"])
        g = np.nonzero(go)[0]
        dxg, dyg, dzg = da[0][h_idx][g], da[1][h_idx][g], da[2][h_idx][g]
        nxg, nyg, nzg = nx[g], ny[g], nz[g]
        k = F(2) * _dot(dxg, dyg, dzg, nxg, nyg, nzg)
        ag = a[g]
        d[0][ag] = dxg - k * nxg
        d[1][ag] = dyg - k * nyg
        d[2][ag] = dzg - k * nzg
        o[0][ag] = hx[g] + BIAS * nxg
        o[1][ag] = hy[g] + BIAS * nyg
        o[2][ag] = hz[g] + BIAS * nzg
        thr[ag] = tt[g] * refl[g]
        alive = ag
    img = np.stack(col, axis=1).astype(F)
    return img, segs
