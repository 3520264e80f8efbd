"""MI355X-native concurrent FIFO queues (G-LFQ, G-WFQ, G-WFQ-YMC) for gfx950.

The queues are hand-written HIP in csrc/, exported through the C ABI of
include/gq.h, include/gq_bench.h, include/gq_serve.h and include/gq_rt.h (libgq.so).  This package is the thin
ctypes binding; importing it loads libgq.so and fails loudly when it is not
built.
"""
from ._binding import (  # noqa: F401
    EXPORTS, GQ_EMPTY, GQ_ERR_CYCLE_BOUND, GQ_ERR_DEVICE, GQ_ERR_HIP, GQ_ERR_INVALID,
    GQ_ERR_NOMEM, GQ_ERR_POOL_EXHAUSTED, GQ_ERR_RESIDENCY, GQ_ERR_TOO_LARGE, GQ_FULL, GQ_OK, KINDS,
    GQError,
    RT_COMPACT, RT_QUEUES, SERVE_HASH_SEED, History, Multi, Queue, RayTracer, Server, Stats, bfs,
    bfs_ctl_bytes,
    device_info, lib, probe_cas,
    probe_copy, probe_faa, probe_fence, required_bytes, resident_blocks, status_str,
)

lib()  # no silent fallback: the HIP library must be present
