"""MI355X (gfx950) library for the modal entropy-stable DG right-hand side of the 2D
shallow water equations on curved triangles (Wu, Kubatko & Chan, arXiv 2005.02516).

* ``binding``   -- ctypes binding of libesdg_swe.so (the C ABI in include/esdg_swe.h)
* ``build``     -- compiles the HIP library in-tree for gfx950
* ``workloads`` -- seeded synthetic meshes, bathymetries and initial states
"""
__all__ = ["binding", "build", "workloads"]
