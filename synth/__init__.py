"""Seeded synthetic inputs for r-cell MD: initial atom states, boxes and deformation paths.

This package holds no arithmetic of the coupling method itself (no QR, no box remap, no
forces, no integration, no stress).  It only draws the inputs that both the FP64 oracle and
the GPU library consume: lattices, random-walk polymer chains, Maxwell-Boltzmann velocities,
random rotations and stretch paths.  Both sides read the same arrays produced here.
"""
from .rng import splitmix64, cell_seed, generator
from .fcc import fcc_lattice
from .kg import kg_melt, kg_box_edge
from .velocities import maxwell_boltzmann
from .deform import (random_rotation, uniaxial_isochoric, rotated_uniaxial, rotated_stretch,
                     stretch_paths, TABLE1_F)
from . import configs

__all__ = ["splitmix64", "cell_seed", "generator", "fcc_lattice", "kg_melt", "kg_box_edge",
           "maxwell_boltzmann", "random_rotation", "uniaxial_isochoric", "rotated_uniaxial",
           "rotated_stretch", "stretch_paths", "TABLE1_F", "configs"]
