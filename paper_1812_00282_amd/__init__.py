"""MI355X-native VATE: sliding-window multi-host cardinality estimation
(Xu, Ding, Hu, arXiv 1812.00282) as hand-written HIP kernels behind a C ABI.

`Sketch` / `Config` (paper_1812_00282_amd.sketch) drive one sketch on the GPU;
`streams` holds the seeded synthetic workloads.  The HIP library libvate.so is
loaded on first use and its absence is an error (no CPU fallback).
"""
__all__ = ["Config", "Sketch"]


def __getattr__(name):
    if name in ("Config", "Sketch"):
        from . import sketch
        return getattr(sketch, name)
    raise AttributeError(name)
