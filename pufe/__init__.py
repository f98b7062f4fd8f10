"""Seeded synthetic PUFE-shaped pencils (H, S): the inputs both the solver and the oracle take."""
from .generate import (Problem, generate, workload, WORKLOADS, guard_vectors, start_block,
                       free_particle_eigs, place_atoms, count_dofs,
                       dof_coordinates, nonlocal_projectors)

__all__ = ["Problem", "generate", "workload", "WORKLOADS", "guard_vectors", "start_block",
           "free_particle_eigs", "place_atoms", "count_dofs", "dof_coordinates", "nonlocal_projectors"]
