"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/*.h declares, and its pure-host logic (sizes,
parameter validation, status strings) behaves as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_01693_amd", "libgq.so")


def declared_functions():
    names = set()
    for h in ("gq.h", "gq_bench.h", "gq_serve.h", "gq_rt.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(gq_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: __graft_entry__.build()"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_binding_signature_table_covers_header():
    from paper_2606_01693_amd import _binding
    assert sorted(_binding.EXPORTS) == sorted(n for n in declared_functions())


def test_library_loads_and_status_strings():
    from paper_2606_01693_amd import _binding as b
    L = b.load_library()
    assert L.gq_status_str(0) == b"ok"
    assert L.gq_status_str(-5).startswith(b"cycle")
    assert L.gq_status_str(99) == b"unknown status"


@pytest.mark.parametrize("cap,width,ok", [
    (1, 8, False), (2, 8, True), (3, 8, False), (1 << 20, 8, True), (1 << 30, 4, True),
    (1 << 31, 8, False), (1024, 2, False), (1024, 4, True),
])
def test_required_bytes_validation(cap, width, ok):
    from paper_2606_01693_amd import _binding as b
    L = b.load_library()
    out = ctypes.c_uint64(0)
    rc = L.gq_required_bytes(0, cap, width, 1, None, ctypes.byref(out))
    assert (rc == 0) == ok
    if ok:
        # two 2n-entry rings of 8-byte words plus n payload cells at least
        assert out.value >= 2 * (2 * cap * 8) + cap * width


def test_required_bytes_padded_layout_is_larger():
    from paper_2606_01693_amd import _binding as b
    compact = b.required_bytes("lfq", 1 << 16, 8, 1, "remap")
    padded = b.required_bytes("lfq", 1 << 16, 8, 1, "padded")
    assert padded - compact >= 2 * (2 << 16) * (128 - 8)


def test_null_arguments_rejected():
    from paper_2606_01693_amd import _binding as b
    L = b.load_library()
    assert L.gq_required_bytes(0, 1024, 8, 1, None, None) == b.GQ_ERR_INVALID
    assert L.gq_destroy(None) == b.GQ_ERR_INVALID
    assert L.gq_create(0, 1024, 8, 1, None, None, 0, None) == b.GQ_ERR_INVALID
    assert L.gq_enqueue_batch(None, None, 0, None, None, None) == b.GQ_ERR_INVALID
    assert L.gq_run_mix(None, 0, 256, 1, None, None, None, None) == b.GQ_ERR_INVALID


def test_wfq_cycle_bound_refused_at_create():
    """Lemma 4: G-WFQ needs R > D*k/n + 6 (R = 2^15 here)."""
    from paper_2606_01693_amd import _binding as b
    # n = 2, D = 64: k = 1023 fits (64*1023 < 32762*2), k = 1024 does not
    assert b.required_bytes("wfq", 2, 8, 1023) > 0
    with pytest.raises(b.GQError) as e:
        b.required_bytes("wfq", 2, 8, 1024)
    assert e.value.status == b.GQ_ERR_CYCLE_BOUND
    # a smaller help delay relaxes the bound
    assert b.required_bytes("wfq", 2, 8, 4000, help_delay=16) > 0
    # lane ids must fit the 20-bit ThrIdx field
    with pytest.raises(b.GQError):
        b.required_bytes("wfq", 1 << 20, 8, 1 << 20)


def test_wfq_layout_includes_records():
    from paper_2606_01693_amd import _binding as b
    lfq = b.required_bytes("lfq", 1 << 12, 8, 4096)
    wfq = b.required_bytes("wfq", 1 << 12, 8, 4096)
    # two rings of 64-byte records per lane plus per-slot owner hints
    assert wfq - lfq >= 2 * 4096 * 64 + 2 * (2 << 12) * 8


@pytest.mark.parametrize("tg,ok", [(0, True), (64, True), (128, True), (1024, True),
                                   (32, False), (96, False), (2048, False)])
def test_ticket_group_validation(tg, ok):
    """The ticket group must be 0 (default) or a power of two in 64..1024."""
    from paper_2606_01693_amd import _binding as b
    if ok:
        assert b.required_bytes("lfq", 1 << 10, 8, 1024, ticket_group=tg) > 0
    else:
        with pytest.raises(b.GQError) as e:
            b.required_bytes("lfq", 1 << 10, 8, 1024, ticket_group=tg)
        assert e.value.status == b.GQ_ERR_INVALID


def test_device_view_struct_matches_header():
    """The ctypes mirror of gq_dev / gq_options has the header's field order."""
    from paper_2606_01693_amd import _binding as b
    hdr = open(os.path.join(ROOT, "include", "gq.h")).read()
    assert "uint32_t ticket_group;" in hdr and "uint32_t group_lanes;" in hdr
    names = [f[0] for f in b._Options._fields_]
    assert names[-1] == "ticket_group"
    dev = [f[0] for f in b._DevView._fields_]
    assert dev[dev.index("help_delay") + 1] == "group_lanes"


@pytest.mark.parametrize("kind,w,h,tile,lanes", [
    (2, 64, 64, 32, 8192),      # G-WFQ-YMC is not offered for the tracer
    (0, 0, 64, 32, 8192),       # empty image
    (0, 64, 64, 24, 8192),      # tile not in {8, 16, 32, 64}
    (0, 64, 64, 32, 1000),      # lanes not a multiple of 256
    (0, 64, 64, 32, 0),
    (1, 64, 64, 32, 1 << 21),   # too many lanes
])
def test_rt_create_rejects_bad_arguments(kind, w, h, tile, lanes):
    """gq_rt_create validates its arguments before touching the device."""
    from paper_2606_01693_amd import _binding as b
    L = b.load_library()
    out = ctypes.c_void_p(0)
    assert L.gq_rt_create(kind, w, h, tile, lanes, ctypes.byref(out)) == b.GQ_ERR_INVALID
    assert out.value is None
    assert L.gq_rt_render(None, None, 0, None, None, None, None) == b.GQ_ERR_INVALID
    assert L.gq_rt_destroy(None) == b.GQ_ERR_INVALID


def test_bfs_static_limits():
    """The allocation-free BFS refuses sizes beyond its fixed maximum before
    any HIP call (no GPU needed), and its static array holds the largest
    configuration: two G-WFQ queues of capacity 2^18 for 8192 lanes plus the
    64 KiB workspace."""
    from paper_2606_01693_amd import _binding
    L = _binding.lib()
    assert L.gq_status_str(-8).startswith(b"size beyond")
    fake = ctypes.c_void_p(4096)
    assert L.gq_bfs_static(0, fake, fake, (1 << 18) + 1, 0, fake, 256, 256, None, None) == -8
    assert L.gq_bfs_static(1, fake, fake, 100, 0, fake, 8192 + 64, 64, None, None) == -8
    assert L.gq_bfs_static(2, fake, fake, 100, 0, fake, 256, 256, None, None) == -1  # YMC
    assert L.gq_bfs_static(0, None, fake, 100, 0, fake, 256, 256, None, None) == -1
    assert L.gq_bfs_static(0, fake, fake, 100, 100, fake, 256, 256, None, None) == -1
    total = 64 * 1024
    for kind in (0, 1):
        b = ctypes.c_uint64(0)
        assert L.gq_required_bytes(kind, 1 << 18, 4, 8192, None, ctypes.byref(b)) == 0
        total_k = 2 * ((b.value + 255) // 256 * 256) + 64 * 1024
        total = max(total, total_k)
    assert total <= 40 << 20
