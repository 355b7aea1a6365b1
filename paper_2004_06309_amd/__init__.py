"""MI355X-native ORAS-preconditioned GMRES for the 3D Helmholtz equation.

``workloads``  seeded synthetic inputs (meshes, velocity models, partitions)
``helm``       ctypes binding of libhelm.so (C-ABI in include/helm.h)
``build``      builds libhelm.so for gfx950
"""
__all__ = ["workloads", "helm", "build"]
