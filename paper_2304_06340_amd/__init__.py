"""MI355X-native H^-s distances between triangulated surfaces.

The computation (exact triangle transforms summed at every node of a
frequency quadrature, residual against the target, Sobolev-weighted
reduction; its NUFFT fast path and adjoint) runs in the HIP kernels of
``libhsd.so``; this package only marshals arguments across the C ABI of
``include/hsd.h``.  Importing the package does not load the library; the
first Context does, and fails loudly if it has not been built.
"""
from .api import (Context, HsdError, Mesh, Params, PointMeasure, Result, Rule, Server, SurfaceMeasure, Ticket,
                  distance, distance_grad, distance_noalloc, transform, transform_rule)

__all__ = ["Context", "HsdError", "Mesh", "Params", "PointMeasure", "Result", "Rule", "Server", "SurfaceMeasure",
           "Ticket",
           "distance", "distance_grad", "distance_noalloc", "transform", "transform_rule"]
