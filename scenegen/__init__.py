"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Holds mesh and scene construction only: no distances, energies, masses or
derivatives of the simulation method live here.
"""
from . import meshes, scenes  # noqa: F401
from .scenes import (CONFIGS, SceneBuilder, default_params, three_cubes,  # noqa: F401
                     icosphere_box, torus_chains, torus_chains_contact, batched_drops, adjoint_drop,
                     near_contact_cubes, triangle_soup, random_state, icosphere_resting_layer,
                     cube_on_slope, sub_scene, cube_lattice, icosphere_fcc, landed,
                     wrecking_ball, hinged_chain, tet_over_ground)
