"""Seeded, synthetic inputs shared by the CPU oracle tests and the GPU path.

This package holds mesh generators, boundary-data generators and inflow
waveforms only.  It contains none of the discretisation's arithmetic (no
residual, stabilisation matrix, transform or solver): both the oracle and the
HIP library receive its arrays as plain inputs.
"""
from .meshgen import (Mesh, cube_kuhn, pipe, junction, boundary_faces,
                      morton_order_elements)
from .problems import (Problem, womersley_problem, junction_problem,
                       cube_problem, initial_guess, tiny_problem,
                       womersley_exact_modes, pipe_family, inlet_waveforms)

__all__ = ["Mesh", "cube_kuhn", "pipe", "junction", "boundary_faces",
           "morton_order_elements", "Problem", "womersley_problem",
           "junction_problem", "cube_problem", "initial_guess",
           "tiny_problem", "womersley_exact_modes", "pipe_family", "inlet_waveforms"]
