"""Host-side check of the segmented contexts (no GPU): the binding refuses
problems that do not share mesh, harmonic count, parameters, Dirichlet node
set and Neumann faces before it creates a context (the library's own
argument checks are in test_abi.py)."""
import pytest

import paper_2311_09465_amd as T
from workloads import womersley_problem
from workloads.meshgen import pipe


def test_segment_solver_rejects_unlike_problems_before_any_device_call():
    mesh = pipe(2, 8)
    a = womersley_problem(K=2, mesh=mesh)
    for b in (womersley_problem(K=3, mesh=mesh),            # other harmonic count
              womersley_problem(K=2, mesh=mesh, Re=50.0),   # other viscosity
              womersley_problem(K=2, mesh=pipe(2, 9))):     # other mesh
        with pytest.raises(T.TsglsError, match="one mesh"):
            T.SegmentSolver.from_problems([a, b])

