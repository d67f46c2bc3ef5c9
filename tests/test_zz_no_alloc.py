"""Allocation-free reduced-basis projection (tsgls_rb_project_noalloc)
against the allocating tsgls_rb_project, through the C ABI.

Both run the same multi-dot and reduction kernels with the same block count,
so the coefficients must agree bit for bit; both are also checked against
the plain FP64 product (Y - mean) Phi^T on the host (1e-12 of the largest
coefficient).  Two calls in a row, the second with a smaller basis and
shorter vectors, so that the fixed scratch array still holds the first
call's partial sums when the second runs."""
import ctypes

import numpy as np
import pytest

from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_noalloc_projection_matches_allocating_projection():
    import torch
    import paper_2311_09465_amd as T
    L = T.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    for case, (N, r, D, seed) in enumerate(((6, 40, 300_001, 1), (3, 7, 1_003, 2))):
        log(f"[gpu] rb_project_noalloc call {case}: N={N} r={r} D={D}")
        rng = np.random.default_rng(seed)
        Phi_h = rng.standard_normal((r, D))
        Y_h = rng.standard_normal((N, D))
        mean_h = rng.standard_normal(D)
        Phi, Y, mean = (torch.from_numpy(a).cuda() for a in (Phi_h, Y_h, mean_h))
        c_alloc = torch.zeros((N, r), dtype=torch.float64, device="cuda")
        c_free = torch.full((N, r), float("nan"), dtype=torch.float64, device="cuda")
        assert L.tsgls_rb_project(P(Phi), r, D, P(Y), N, P(mean), P(c_alloc), stream) == 0
        assert L.tsgls_rb_project_noalloc(P(Phi), r, D, P(Y), N, P(mean), P(c_free), stream) == 0
        torch.cuda.synchronize()
        a, b = c_alloc.cpu().numpy(), c_free.cpu().numpy()
        ref = (Y_h - mean_h) @ Phi_h.T
        err = np.abs(b - ref).max() / np.abs(ref).max()
        log(f"[gpu]   bitwise equal: {np.array_equal(a, b)}; rel err vs host FP64 {err:.2e}")
        assert np.array_equal(a, b)
        assert err <= 1e-12
    # more basis vectors than the scratch holds: rejected before any device work
    assert L.tsgls_rb_project_noalloc(P(Phi), 1025, D, P(Y), N, P(mean), P(c_free), stream) == -7
