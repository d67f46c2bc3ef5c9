"""Oracle solve against the Womersley closed form (the consistency case:
u . grad u = 0 exactly for pulsatile pipe flow, whose solution is unique as
the remark on existence and uniqueness notes).  Pipe R = 1, L = 4, Re = 100,
Wo = 5, inlet flow Qbar (1 + 0.5 sin(omega t)), exact inlet profile per mode,
no-slip wall, zero-traction outlet.  The velocity error must fall at a rate
of at least 1.5 between two refinements (rate 2 expected in the diffusive
regime, 1.5 in the convective one)."""
import numpy as np
import pytest

import oracle as O
from workloads import womersley_problem, initial_guess


def _err(nr, nl):
    prob = womersley_problem(nr, nl, K=1)
    par = O.Params.from_problem(prob)
    y, st = O.solve(par, prob.mesh.xyz, prob.mesh.tets, initial_guess(prob),
                    rtol=1e-7, variant="picard")
    assert st["rel_residual"] <= 1e-7
    ex = prob.exact
    return np.linalg.norm(y[:, :3] - ex[:, :3]) / np.linalg.norm(ex[:, :3])


@pytest.mark.slow
def test_womersley_convergence():
    e1 = _err(2, 8)
    e2 = _err(4, 16)
    rate = np.log2(e1 / e2)
    assert e2 < 0.03
    assert rate >= 1.5, (e1, e2, rate)
