"""Seeded synthetic inputs (pocket grids, random-tree ligand libraries, start
orientations) shared by the oracle tests, the GPU tests and the benchmark.

This module makes inputs only; it contains no docking arithmetic.
"""
from .synth import (  # noqa: F401
    Library,
    Pocket,
    PocketAtoms,
    pocket_atoms,
    build,
    library_uniform,
    library_lognormal,
    library_from_sizes,
    pocket_gaussians,
    start_quats,
    config,
    CONFIGS,
    MASTER_SEED,
)
