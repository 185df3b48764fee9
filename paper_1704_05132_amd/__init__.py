"""MI355X-native VNS for the uncapacitated multi-item economic lot-sizing problem with remanufacturing.

The search runs in hand-written HIP kernels behind the C ABI of include/vns.h (libvns.so); `vns` is its
thin Python binding and `instances` draws seeded synthetic instances.
"""
__all__ = ["instances", "vns"]
