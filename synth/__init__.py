"""Seeded synthetic inputs for the plane-wave H*psi path.

This package builds the *workload*: cells, plane-wave spheres, FFT boxes,
local potentials sampled on the grid, Kleinman-Bylander projector tables and
random start blocks.  It holds none of the method's arithmetic (no FFT, no
Hamiltonian application, no filter, no subspace step); both the CPU oracle
and the GPU library receive its arrays as inputs.
"""
from .cells import (  # noqa: F401
    Cell, Workload, diamond_cell, make_workload, sphere_miller, box_rule,
    local_potential, kb_projectors, start_block, kpoint_grid_shifted,
    config_c1, config_c2, config_c3, config_c4, config_c5, c4_cell_params, CONFIGS,
)
