"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no part of the method's arithmetic (no Fourier transform,
no quadrature, no reduction).  It only builds the *inputs* the method is run
on: icosahedral triangulations of the unit sphere (the paper's test surfaces,
Section 4.2), their stretches onto ellipsoids, grid triangulations of tori,
radial perturbations and rigid rotations of them, random
triangles and frequency points for unit tests, and the Poisson request trace
used by the serving benchmark.  Every generator takes an explicit seed or
``numpy.random.Generator`` so that the GPU path and the oracle see bit-identical
arrays.
"""
from .meshes import (icosahedron, icosphere, mean_edge_length, perturb_radial,
                     perturb_harmonic, random_rotation, rotate, random_triangles,
                     random_points, icosphere_counts, ellipsoid_mesh, torus_mesh)
from .trace import serving_trace, Request

__all__ = [
    "icosahedron", "icosphere", "icosphere_counts", "mean_edge_length",
    "perturb_radial", "perturb_harmonic", "random_rotation", "rotate",
    "random_triangles", "random_points", "serving_trace", "Request",
    "ellipsoid_mesh", "torus_mesh",
]
