"""MI355X-native partitioned single-source shortest paths (SP-Async hot path).

Submodules are imported on demand: ``gen`` (seeded synthetic inputs) and
``sssp`` (the ctypes binding over the HIP library).
"""
__all__ = ["gen", "sssp"]
