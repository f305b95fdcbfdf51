"""Seeded synthetic inputs for the wall-modeled IBM stage.

This package only builds input data: staggered grids, signed-distance
fields of terrains, velocity, sub-grid stress and pressure-gradient fields.
It holds none of the method's arithmetic (no classification, no wall
model, no divergence, no forcing), so that the CPU reference and the GPU
library can both be fed from it without sharing any of the computation
they are compared on.
"""
from .grid import Grid, node_z, node_xy
from . import terrain, fields, configs

__all__ = ["Grid", "node_z", "node_xy", "terrain", "fields", "configs"]
