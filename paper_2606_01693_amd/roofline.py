"""Roofline probes for the queue kernels on one GPU.

Measures, with HIP events on the current stream:
  - R_ctr: WaveFAA rate on 1..16 counters (same-address atomic throughput);
  - agent-scope release / acquire fence cost with every wavefront fencing;
  - R_slot: 64-bit CAS rate on distinct slots at several strides;
and prints one line per measurement.  Usage: python -m paper_2606_01693_amd.roofline
"""
from __future__ import annotations


def _timed(torch, fn, reps=3):
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def main():
    import torch

    from . import _binding as gq

    torch.cuda.set_device(0)
    buf = torch.zeros((64 << 20) // 8, dtype=torch.int64, device="cuda")
    lanes = 2048 * 256
    for nc in (1, 2, 4, 8, 16):
        for sp in (256, 4096, 65536, 1 << 20):
            gq.probe_faa(buf, lanes, 2, False, nc, sp)
            ms = _timed(torch, lambda: gq.probe_faa(buf, lanes, 32, False, nc, sp))
            rate = (lanes // 64) * 32 / (ms * 1e-3)
            print(f"faa_wave nc={nc:2d} sp={sp:8d}: {rate / 1e6:9.1f} M FAA/s total, "
                  f"{rate / nc / 1e6:8.1f} per counter", flush=True)
    for lanes2 in (256 * 64, 256 * 256, 2048 * 256):
        ms = _timed(torch, lambda: gq.probe_faa(buf, lanes2, 32, False, 1, 256))
        print(f"faa_wave single counter lanes={lanes2}: {(lanes2 // 64) * 32 / (ms * 1e-3) / 1e6:.1f} M/s",
              flush=True)
    lines = torch.zeros(lanes // 64 * 32, dtype=torch.int64, device="cuda")
    for mode in (0, 1, 2, 3):
        gq.probe_fence(lines, lanes, 2, mode)
        ms = _timed(torch, lambda: gq.probe_fence(lines, lanes, 64, mode))
        print(f"fence mode={mode}: {ms:.3f} ms for 64 iters x {lanes // 64} waves -> "
              f"{ms * 1e6 / 64:.1f} ns per iter (all waves)", flush=True)
    nslots = 2 << 20
    for stride in (8, 64, 128, 256):
        slots = torch.zeros(nslots * stride // 8, dtype=torch.int64, device="cuda")
        gq.probe_cas(slots, nslots, stride, lanes, 2)
        ms = _timed(torch, lambda: gq.probe_cas(slots, nslots, stride, lanes, 16))
        print(f"cas stride={stride}: {lanes * 16 / (ms * 1e-3) / 1e9:.2f} G CAS/s", flush=True)
        del slots


if __name__ == "__main__":
    main()
