"""covox on MI355X: projective or raycast TSDF integration into a voxel-hashed block grid,
the exact ESDF derived from it, and correspondence-free ESDF submap alignment
(Hoss and De Cristoforis, coVoxSLAM, arXiv 2410.21149), as hand-written HIP
kernels for gfx950 behind the C ABI in include/covox.h.

``Context`` wraps a library context; importing this package fails when the
HIP library has not been built.
"""
from .covox import (AlignSet, EDEGENERATE, EHIP, EINVAL, EPOOL_FULL, ESDF_EXACT, ESDF_WAVEFRONT, ETABLE_FULL, FP16, FP32,
                    GAUSS_NEWTON, KERNELS, LEVENBERG_MARQUARDT, LIB_PATH, NET_NOALLOC_MAX_PAIRS, NOT_CONVERGED, OK,
                    PROJECTIVE, RAYCAST, WEIGHT_CONSTANT, WEIGHT_INV_DEPTH2, Context, CovoxError, Graph, Net, Submap,
                    default_params)

__all__ = ["AlignSet", "Context", "Graph", "Net", "Submap", "CovoxError", "default_params", "FP32", "FP16", "WEIGHT_CONSTANT",
           "WEIGHT_INV_DEPTH2", "PROJECTIVE", "RAYCAST", "ESDF_EXACT", "ESDF_WAVEFRONT",
           "GAUSS_NEWTON", "LEVENBERG_MARQUARDT", "KERNELS", "OK", "EINVAL",
           "EPOOL_FULL", "ETABLE_FULL", "EHIP", "EDEGENERATE", "NOT_CONVERGED", "LIB_PATH", "NET_NOALLOC_MAX_PAIRS"]
