"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds no part of the density-fitted J/K arithmetic.  It only
draws random numbers and builds the problem description: water-cluster
geometries, the uncontracted spherical AO and auxiliary basis sets, occupied
orbital coefficients (orthonormal in the AO overlap, which it evaluates by
brute-force quadrature of the basis functions themselves) and request streams.
"""
from .water import (  # noqa: F401
    ANGSTROM_TO_BOHR,
    Molecule,
    water_monomer,
    water_cluster,
    make_molecule,
    overlap_by_quadrature,
    occupied_orbitals,
    perturbed_orbitals,
    poisson_stream,
    config,
    cluster_box,
    build_case,
    shift_molecule,
)
