"""Pins for the modal representation and the convolution matrix.

The oracle's Toeplitz product A(u) c (eq. phi-def) must equal the truncated
product of the two real periodic signals, computed here independently by a
finely sampled FFT.  The dealiasing facts the HIP path relies on (3K+1
samples reproduce the truncated product exactly, 3K do not) are checked
against the same oracle matrix.
"""
import numpy as np
import pytest

import oracle as O


def _rand_modes(rng, K, shape=()):
    y = rng.standard_normal(shape + (2 * K + 2,))
    y[..., 1] = 0.0
    return O.slots_to_modes(y, K)


def _signal(c, t, omega=1.0):
    K = (c.shape[-1] - 1) // 2
    m = np.arange(-K, K + 1)
    return (c[..., None, :] * np.exp(1j * omega * np.outer(t, m))).sum(-1).real


@pytest.mark.parametrize("K", [0, 1, 3, 6, 15])
def test_toeplitz_is_truncated_product(K):
    rng = np.random.default_rng(K)
    u, c = _rand_modes(rng, K), _rand_modes(rng, K)
    Msamp = 8 * (K + 1) + 1
    t = 2 * np.pi * np.arange(Msamp) / Msamp
    prod = _signal(u, t) * _signal(c, t)
    coef = np.fft.fft(prod) / Msamp                       # coef[k] = mode k
    ref = np.array([coef[m % Msamp] for m in range(-K, K + 1)])
    got = O.toeplitz(u) @ c
    assert np.allclose(got, ref, atol=1e-13 * max(1, np.abs(ref).max()))
    A = O.toeplitz(u)
    assert np.allclose(A, A.conj().T)                    # Hermitian for real u


@pytest.mark.parametrize("K", [1, 3, 6, 15, 31])
def test_dealiased_sampling_exact_at_3K_plus_1(K):
    rng = np.random.default_rng(100 + K)
    u, c = _rand_modes(rng, K), _rand_modes(rng, K)
    ref = O.toeplitz(u) @ c
    m = np.arange(-K, K + 1)

    def sampled(M):
        t = 2 * np.pi * np.arange(M) / M
        f = _signal(u, t) * _signal(c, t)
        return np.array([(f * np.exp(-1j * mm * t)).sum() / M for mm in m])

    err_ok = np.abs(sampled(3 * K + 1) - ref).max() / np.abs(ref).max()
    err_bad = np.abs(sampled(3 * K) - ref).max() / np.abs(ref).max()
    assert err_ok < 1e-13
    assert err_bad > 1e-6          # the bound M >= 3K+1 is tight


def test_slots_roundtrip_and_im0_ignored():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((5, 4, 8))
    c = O.slots_to_modes(y, 3)
    assert np.allclose(c[..., 3].imag, 0.0)
    back = O.modes_to_slots(c, 3)
    yy = y.copy()
    yy[..., 1] = 0
    assert np.allclose(back, yy)
    # conjugate symmetry
    assert np.allclose(c[..., :3][..., ::-1], np.conj(c[..., 4:]))
