/* gq_rt.h -- tile-based wavefront ray tracer driven by the device queues.
 *
 * The paper's ray-tracing workload (Section V-B, tile-based wavefront ray
 * tracing; results in Section VI-E): a W x H image is cut into square tiles,
 * each tile owns one queue, primary rays are enqueued per tile, and a
 * persistent kernel dequeues work, traces and shades one path segment, and
 * re-enqueues the reflective bounce into the same tile's queue until no work
 * remains.  Here a wavefront claims one tile at a time from a global cursor
 * and works its queue until a dequeue of all its lanes finds it empty.  It is
 * compared with a stream-compaction tracer that gathers the surviving rays
 * into a dense list between passes, one launch per bounce depth.
 *
 * What is traced (both methods compute the same bits per pixel): the path of
 * each pixel, segment by segment, in float32, each operation rounded in a
 * fixed order:
 *   primary ray: o = eye, d = v * (1 / sqrt(v.v)) with
 *     v = ((x + 0.5) sx - ax, ay - (y + 0.5) sy, -1)
 *   per segment: nearest of the spheres (index order; oc = o - c, b = oc.d,
 *     q = oc.oc - r2, disc = b*b - q, t = (-b) - sqrt(disc), or (-b) + sqrt(disc)
 *     when that is <= 1e-4) and then the planes (den = n.d < 0,
 *     t = (d_plane - n.o) / den), candidates need t > 1e-4 and strictly beat
 *     the best so far; a dot product is ((x0*y0) + (x1*y1)) + (x2*y2)
 *   miss: colour += thr * background, path ends
 *   hit at h = o + t*d, normal n (sphere (h - c) * inv_r, plane n):
 *     colour_c += (thr * albedo_c) * (ambient + diffuse * max(0, n.L));
 *     with refl > 0 and depth < max_bounces: d = d - (2 (d.n)) n,
 *     o = h + 1e-3 n, thr *= refl, depth += 1, next segment; else the path ends
 *
 * Queue kinds: G-LFQ and G-WFQ (G-WFQ-YMC is not offered here: its memory
 * grows with every poll of an empty tile queue).
 */
#ifndef GQ_RT_H
#define GQ_RT_H

#include <stdint.h>

#include "gq.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GQ_RT_MAX_SPHERES 128u
#define GQ_RT_MAX_PLANES 8u

typedef struct gq_rt_scene {
    const float *spheres;   /* device, n_spheres x 10: cx cy cz r2 inv_r albedo_rgb refl pad */
    const float *planes;    /* device, n_planes x 8: nx ny nz d albedo_rgb refl (n.p = d,
                               unit normal facing the scene)                            */
    uint32_t n_spheres;     /* <= GQ_RT_MAX_SPHERES                                      */
    uint32_t n_planes;      /* <= GQ_RT_MAX_PLANES                                       */
    float camera[7];        /* eye x y z, sx, sy, ax, ay (see above)                     */
    float light[3];         /* unit vector towards the directional light                */
    float shade[2];         /* ambient, diffuse                                          */
    float background[3];
    uint32_t max_bounces;   /* <= 16                                                     */
} gq_rt_scene;

typedef enum { GQ_RT_QUEUES = 0, GQ_RT_COMPACT = 1 } gq_rt_method;

typedef struct gq_rt gq_rt;

/* Create a tracer for width x height images cut into tile x tile tiles
 * (tile 8, 16, 32 or 64; edge tiles are partial).  `kind` is the tile queues'
 * kind (GQ_LFQ or GQ_WFQ), one queue of capacity tile^2 per tile; `lanes` is
 * the persistent kernel's lane count (a multiple of 256, at most 2^20).  The
 * library allocates the queues, the per-pixel path state (11 words per pixel)
 * and the compaction lists; gq_rt_destroy frees them.  Errors: GQ_ERR_INVALID
 * for a bad size, tile, kind or lane count, GQ_ERR_NOMEM / GQ_ERR_HIP from the
 * runtime, GQ_ERR_CYCLE_BOUND when G-WFQ refuses the lane count per queue. */
gq_status gq_rt_create(gq_kind kind, uint32_t width, uint32_t height, uint32_t tile,
                       uint32_t lanes, gq_rt **out);

/* Render `scene` with `method` on `stream` (stream-ordered, asynchronous).
 * d_image: device float[width * height * 3], row-major RGB, fully written.
 * d_segments: device uint32[width * height] or NULL: segments traced per pixel.
 * d_stats: device uint64[4] or NULL, overwritten: {segments traced, bounce
 *   re-enqueues, dequeues that found a tile empty, launches}.
 * The queue method ends when every path has ended; a run still going after
 * 10 s of the GPU clock latches GQ_ERR_DEVICE (read with gq_rt_check_error)
 * instead of running on.  Scene arrays stay owned by the caller and must stay
 * valid until the work on `stream` is done. */
gq_status gq_rt_render(gq_rt *rt, const gq_rt_scene *scene, uint32_t method, float *d_image,
                       uint32_t *d_segments, uint64_t *d_stats, void *stream);

/* Latched device error of the last render (GQ_OK if none); synchronizes `stream`.
 * A queue render that ended with a path still unfinished also reports
 * GQ_ERR_DEVICE; after any error the next queue render resets the tile queues
 * first. */
gq_status gq_rt_check_error(gq_rt *rt, void *stream);

gq_status gq_rt_destroy(gq_rt *rt);

#ifdef __cplusplus
}
#endif

#endif /* GQ_RT_H */
