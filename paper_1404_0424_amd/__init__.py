"""CG soft-output MMSE detection and CG precoding for massive MIMO on MI355X.

Kernels are hand-written HIP for gfx950 in libmimocg.so (C ABI in
include/mimo_cg.h).  ``api`` is the torch binding; ``workload`` draws seeded
synthetic inputs.  Submodules are imported on demand so that the input
generator can be used without loading the GPU library.
"""
__all__ = ["api", "workload", "build", "serving"]
